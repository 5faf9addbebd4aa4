// Transforms between the plane-wave sphere and the real-space grid, the
// pair-density Poisson solves and the exchange contraction.
//
// Paper mapping (Sec. 2.1 and Sec. 3.2):
//  * sphere <-> real space: the orbital and trial-vector FFTs;
//  * pairs_to_dsticks + dstick_poisson + dsticks_to_fields: the pair potentials
//    tau_vv' = v_c * (phi_v phi_v') of Eq. trunc (the N_occ^2 integrations) and
//    the Hartree part of f_Hxc in Eq. k1eterm;
//  * contract: R_v = c_K phi_v (v_H + f_xc drho) - alpha sum_v' tau_vv' a_v'
//    (the K1e and K1d integrands of Eqs. k1eterm and k1d before projection).
//
// Real fields are stored as f[(i0*n1 + i1)*n2 + i2].  A 3D transform is a
// stick pass (1D FFTs along i0 of the columns (k1, k2) that can be nonzero)
// and a plane pass (2D FFT over (i1, i2) at fixed i0, staged in LDS).  Two real
// fields travel as the real and imaginary parts of one complex field (the
// Gamma-point packing).  Stick data layout: [pack][i0 or k0][stick].
#include <algorithm>

#include "wtd_fft_ct.h"
#include "wtd_fft_reg.h"
#include "wtd_internal.h"

namespace wtd {

namespace {

constexpr int kStickThreads = 256;
constexpr int kPlaneThreads = 512;
constexpr int kPairItems = 4;  // (plane, pack) items per workgroup of the prefetching pair kernel
constexpr int kStickRegs = 6;  // rounds of density-stick loads held in registers by the plane kernels
// wave sticks per thread of the compile-time plane kernels (577 sticks at
// 72^3 / 40 Ry, 1,305 at 108^3)
template <int SN>
constexpr int wave_stick_regs() {
  return SN >= 96 ? 3 : 2;
}
// (108 x 108 planes run one workgroup per CU, so they keep every round of the
// 108^3 density sticks in registers)
template <int SN>
constexpr int stick_regs() {
  return SN == 108 ? 11 : kStickRegs;
}

// items per workgroup of the pair-product kernel: kPairItems for FP64 planes up
// to 72 x 72 (compile-time plans), one otherwise
template <int SN, typename T>
constexpr int pair_items() {
  return (SN > 0 && SN * SN <= 72 * 72 && sizeof(T) == 8) ? kPairItems : 1;
}

// items per workgroup of the inverse group kernel: FP64 planes take one
// workgroup per CU, whose next item's loads are then hidden by prefetch (72^3
// FP64 inverse pass 13.3 ms per apply with one item, 12.1 with 2, 11.5 with 4);
// FP32 keeps one item and three workgroups per CU (6.5 ms against 4.5 with 2)
constexpr int kGroupItems = 4;
template <typename T>
constexpr int group_items() {
  return sizeof(T) == 8 ? kGroupItems : 1;
}

int min_radix(const FFTPlan& p) {
  int r = 8;
  for (int i = 0; i < p.np; ++i) r = p.rad[i] < r ? p.rad[i] : r;
  return r;
}

int pick_maxb(int nlines, const FFTPlan& p, int nthreads) {
  int64_t total = (int64_t)nlines * (p.n / min_radix(p));
  int64_t need = (total + nthreads - 1) / nthreads;
  if (need <= 1) return 1;
  if (need <= 2) return 2;
  if (need <= 4) return 4;
  if (need <= 8) return 8;
  throw StatusError{WTD_ERR_SHAPE, "FFT line batch too large for one workgroup"};
}

#define WTD_MAXB_DISPATCH(maxb, ...)                              \
  switch (maxb) {                                                 \
    case 1: { constexpr int MB = 1; __VA_ARGS__; } break;         \
    case 2: { constexpr int MB = 2; __VA_ARGS__; } break;         \
    case 4: { constexpr int MB = 4; __VA_ARGS__; } break;         \
    default: { constexpr int MB = 8; __VA_ARGS__; } break;        \
  }

// 2D FFT of the LDS plane [k1][k2] (k2 fastest): S = -1 rows first then columns
// (forward), S = +1 columns first then rows (inverse).  SN > 0: n1 = n2 = SN with
// a compile-time plan and the twiddle table `twl` in LDS, the column pass on
// the columns of P1.cut only; SN = 0: runtime plans, every column.
template <int S, int SN, int MB1, int MB2, typename T>
__device__ __forceinline__ void plane_fft(cplx<T>* pl, const FFTPlan& P1, const FFTPlan& P2,
                                          int n1, int n2, const cplx<T>* tw1,
                                          const cplx<T>* tw2, const cplx<T>* twl) {
  if constexpr (SN > 0) {
    // the columns outside P1.cut hold nothing the caller reads (forward) or
    // only zeros (inverse)
    if (S < 0) {
      ct_fft<S, SN, SN, 1, SN, kPlaneThreads, false>(pl, twl);
      ct_fft_cols<S, SN, kPlaneThreads>(pl, twl, P1.cut);
    } else {
      ct_fft_cols<S, SN, kPlaneThreads>(pl, twl, P1.cut);
      ct_fft<S, SN, SN, 1, SN, kPlaneThreads, false>(pl, twl);
    }
  } else {
    if (S < 0) {
      lds_fft<S, MB2, false>(pl, P2, n1, 1, n2, tw2);   // along i2: n1 rows
      lds_fft<S, MB1, true>(pl, P1, n2, n2, 1, tw1);    // along i1: n2 columns
    } else {
      lds_fft<S, MB1, true>(pl, P1, n2, n2, 1, tw1);
      lds_fft<S, MB2, false>(pl, P2, n1, 1, n2, tw2);
    }
  }
}

// 1D FFTs along i0 of kStickTile sticks held as [i0][stick] in LDS.
template <int S, int SN, int MB, typename T>
__device__ __forceinline__ void stick_fft(cplx<T>* buf, const FFTPlan& P0, const cplx<T>* tw0,
                                          const cplx<T>* twl) {
  if constexpr (SN > 0)
    ct_fft<S, SN, kStickTile, kStickTile, 1, kStickThreads, true>(buf, twl);
  else
    lds_fft<S, MB, true>(buf, P0, kStickTile, kStickTile, 1, tw0);
}

// Workgroups are dealt to the 8 XCDs round-robin by linear id.  xcd_item maps a
// linear id to a work item so that each XCD walks a contiguous range of items:
// items sharing inputs then meet in the same L2.  Returns -1 for the padding ids.
__device__ __forceinline__ int xcd_item(int total) {
  const int per = (total + 7) >> 3;
  const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  return w < total ? w : -1;
}

// copy an N-entry twiddle table into LDS (callers synchronise before use)
template <int SN, typename T>
__device__ __forceinline__ void stage_twiddles(cplx<T>* twl, const cplx<T>* tw) {
  if constexpr (SN > 0)
    for (int i = threadIdx.x; i < SN; i += blockDim.x) twl[i] = tw[i];
}

// ---------------------------------------------------------------- sphere -> sticks
// coef: [nb][per_trial][npw][2]; pack (b, j) carries fields v = 2j (re) and 2j+1 (im).
template <int MB, int SN, typename T>
__global__ void __launch_bounds__(kStickThreads)
k_sphere_to_wsticks(const T* __restrict__ coef, int per_trial, int npt, int npw, int n0, int nw,
                    int nws,
                    const int* __restrict__ off, const int4* __restrict__ ent, FFTPlan P0,
                    const cplx<T>* __restrict__ tw0, cplx<T>* __restrict__ wst) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tile = blockIdx.x;
  const int pack = blockIdx.y;
  const int b = pack / npt, j = pack - b * npt;
  const int v1 = 2 * j, v2 = 2 * j + 1;
  const T* c1 = coef + ((int64_t)b * per_trial + v1) * npw * 2;
  const T* c2 = (v2 < per_trial) ? c1 + (int64_t)npw * 2 : nullptr;
  const int tot = n0 * kStickTile;
  cplx<T>* twl = buf + tot;
  stage_twiddles<SN>(twl, tw0);
  for (int i = threadIdx.x; i < tot; i += blockDim.x) buf[i] = {T(0), T(0)};
  __syncthreads();
  for (int e = off[tile] + threadIdx.x; e < off[tile + 1]; e += blockDim.x) {
    const int4 q = ent[e];  // (h, sign, local stick, k0)
    const int h = q.x;
    T ar = c1[2 * h], ai = c1[2 * h + 1];
    T br = c2 ? c2[2 * h] : T(0), bi = c2 ? c2[2 * h + 1] : T(0);
    cplx<T> z;
    if (h == 0) {
      z = {ar, br};
    } else if (q.y > 0) {
      z = {ar - bi, ai + br};          // c1(m) + i c2(m)
    } else {
      z = {ar + bi, br - ai};          // conj(c1(m)) + i conj(c2(m))
    }
    buf[q.w * kStickTile + q.z] = z;
  }
  __syncthreads();
  stick_fft<+1, SN, MB>(buf, P0, tw0, twl);
  cplx<T>* out = wst + (int64_t)pack * n0 * nws;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) {
    const int i0 = i / kStickTile, l = i - i0 * kStickTile;
    const int s = tile * kStickTile + l;
    if (s < nw) out[(int64_t)i0 * nws + s] = buf[i];
  }
}

// ---------------------------------------------------------------- sticks -> real fields
// One workgroup per (i0, trial b); loops over the packs of that trial.  With
// drho != nullptr also forms drho_b = sum_v phi_v out_bv on the plane.
// (FP32 on 72 x 72 planes: capped at 128 registers so two workgroups share a CU,
// as the LDS allows)
template <int MB1, int MB2, int SN, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
__attribute__((amdgpu_waves_per_eu((SN == 72 && sizeof(T) == 4) ? 4 : 1)))
k_wsticks_to_fields(const cplx<T>* __restrict__ wst, int npt, int per_trial, int n0, int n1,
                    int n2, int nw, int nws, const int* __restrict__ k12, FFTPlan P1, FFTPlan P2,
                    const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2, T scale,
                    T* __restrict__ out, const T* __restrict__ phi, T* __restrict__ drho,
                    int ngroup, int nbtot) {
  extern __shared__ unsigned char smem_raw[];
  const int plane = n1 * n2;
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  // the density accumulator: in LDS behind the plane for runtime plans, in
  // registers (each thread always owns the same points) for compile-time ones
  T* acc = reinterpret_cast<T*>(pl + plane);
  cplx<T>* twl = reinterpret_cast<cplx<T>*>(acc + ((drho && SN == 0) ? plane : 0));
  // item = (i0, group, b), b fastest: the trials of one (plane, orbital group)
  // read the same orbital planes and run back to back on one XCD.  The packs
  // of trial b are split into ngroup contiguous groups; each group writes its
  // own partial drho.
  const int item = xcd_item(n0 * ngroup * nbtot);
  if (item < 0) return;
  stage_twiddles<SN>(twl, tw1);
  const int i0 = item / (ngroup * nbtot);
  const int rem = item - i0 * ngroup * nbtot;
  const int grp = rem / nbtot, b = rem - grp * nbtot;
  const int per = (npt + ngroup - 1) / ngroup;
  const int j0 = grp * per, j1 = min(npt, j0 + per);
  const int64_t nr = (int64_t)n0 * plane;
  const int64_t poff = (int64_t)i0 * plane;
  if constexpr (SN > 0) {
    // the next pack's sticks and the current pack's orbital planes are loaded
    // into registers before the plane FFT, so their latency overlaps it
    constexpr int PL = SN * SN;
    constexpr int EL = (PL + kPlaneThreads - 1) / kPlaneThreads;
    constexpr int WS = wave_stick_regs<SN>();  // nw <= WS * kPlaneThreads, host-checked
    T racc[EL];
#pragma unroll
    for (int e = 0; e < EL; ++e) racc[e] = T(0);
    cplx<T> sv[WS];
    int kv[WS];
#pragma unroll
    for (int e = 0; e < WS; ++e) {
      const int st = threadIdx.x + e * kPlaneThreads;
      kv[e] = st < nw ? k12[st] : -1;
    }
    auto load_sticks = [&](int j) {
      const cplx<T>* src = wst + ((int64_t)(b * npt + j) * n0 + i0) * nws;
#pragma unroll
      for (int e = 0; e < WS; ++e)
        if (kv[e] >= 0) sv[e] = src[threadIdx.x + e * kPlaneThreads];
    };
    if (j0 < j1) load_sticks(j0);
    for (int j = j0; j < j1; ++j) {
      for (int i = threadIdx.x; i < plane; i += blockDim.x) pl[i] = {T(0), T(0)};
      __syncthreads();
#pragma unroll
      for (int e = 0; e < WS; ++e)
        if (kv[e] >= 0) pl[kv[e]] = sv[e];
      __syncthreads();
      if (j + 1 < j1) load_sticks(j + 1);
      const int v1 = 2 * j, v2 = 2 * j + 1;
      const bool has2 = v2 < per_trial;
      T f1[EL], f2[EL];
      if (drho) {
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          const int i = threadIdx.x + e * kPlaneThreads;
          if (PL % kPlaneThreads == 0 || i < PL) {
            f1[e] = phi[(int64_t)v1 * nr + poff + i];
            f2[e] = has2 ? phi[(int64_t)v2 * nr + poff + i] : T(0);
          }
        }
      }
      plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
      T* o1 = out + ((int64_t)b * per_trial + v1) * nr + poff;
      T* o2 = o1 + nr;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) {
          const cplx<T> z = pl[i];
          const T a = z.x * scale, c = z.y * scale;
          o1[i] = a;
          if (has2) o2[i] = c;
          if (drho) racc[e] += f1[e] * a + f2[e] * c;
        }
      }
      __syncthreads();
    }
    if (drho) {
      T* d = drho + ((int64_t)grp * nbtot + b) * nr + poff;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) d[i] = racc[e];
      }
    }
  } else {
  if (drho)
    for (int i = threadIdx.x; i < plane; i += blockDim.x) acc[i] = T(0);
  for (int j = j0; j < j1; ++j) {
    const int pack = b * npt + j;
    for (int i = threadIdx.x; i < plane; i += blockDim.x) pl[i] = {T(0), T(0)};
    __syncthreads();
    const cplx<T>* src = wst + ((int64_t)pack * n0 + i0) * nws;
    for (int s = threadIdx.x; s < nw; s += blockDim.x) pl[k12[s]] = src[s];
    __syncthreads();
    plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
    const int v1 = 2 * j, v2 = 2 * j + 1;
    T* o1 = out + ((int64_t)b * per_trial + v1) * nr + poff;
    T* o2 = o1 + nr;
    const bool has2 = v2 < per_trial;
    for (int i = threadIdx.x; i < plane; i += blockDim.x) {
      const cplx<T> z = pl[i];
      const T a = z.x * scale, c = z.y * scale;
      o1[i] = a;
      if (has2) o2[i] = c;
      if (drho) {
        T d = phi[(int64_t)v1 * nr + poff + i] * a;
        if (has2) d += phi[(int64_t)v2 * nr + poff + i] * c;
        acc[i] += d;
      }
    }
    __syncthreads();
  }
  if (drho) {
    T* d = drho + ((int64_t)grp * nbtot + b) * nr + poff;
    for (int i = threadIdx.x; i < plane; i += blockDim.x) d[i] = acc[i];
  }
  }
}

// drho[b] = sum over groups of the partial densities (fixed order)
template <typename T>
__global__ void k_sum_groups(const T* __restrict__ part, int ngroup, int64_t n,
                             T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = T(0);
  for (int gr = 0; gr < ngroup; ++gr) s += part[(int64_t)gr * n + i];
  out[i] = s;
}

// ---------------------------------------------------------------- pair products -> density sticks
// quad (a, b, c, d): re = src[a]*src[b] (or src[a] if b < 0), im likewise from (c, d);
// c < 0 means no imaginary part.
template <int MB1, int MB2, int SN, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_pairs_to_dsticks(const T* __restrict__ src, const int4* __restrict__ quads, int npack, int limit,
                   int n0,
                   int n1, int n2, int nd, int nds, const int* __restrict__ k12, FFTPlan P1,
                   FFTPlan P2,
                   const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                   cplx<T>* __restrict__ dst) {
  extern __shared__ unsigned char smem_raw[];
  const int plane = n1 * n2;
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* twl = pl + plane;
  const int64_t nr = (int64_t)n0 * plane;
  // item = (i0, pack), pack fastest: an XCD works through its planes one at a
  // time, so the orbital planes of the current i0 stay in its L2
  const int total = n0 * npack;
  if constexpr (pair_items<SN, T>() > 1) {
    // kPairItems consecutive items per workgroup; the four orbital planes of
    // the next item are loaded into registers while the current one is
    // transformed (FP64: one workgroup per CU fits the LDS, so the latency of
    // the next item's loads is hidden by prefetch instead of by other
    // workgroups; FP32 keeps one item per workgroup and three workgroups per CU)
    constexpr int PL = SN * SN;
    constexpr int EL = (PL + kPlaneThreads - 1) / kPlaneThreads;
    const int grp = xcd_item((total + kPairItems - 1) / kPairItems);
    if (grp < 0) return;
    stage_twiddles<SN>(twl, tw1);
    const int it0 = grp * kPairItems, it1 = min(total, it0 + kPairItems);
    T ra[EL], rb[EL], rc[EL], rd[EL];
    auto load = [&](int item) {
      const int i0 = item / npack;
      const int pack = item - i0 * npack;
      const int64_t poff = (int64_t)i0 * plane;
      int4 q = quads[pack];
      if (q.z >= limit) q.z = -1;  // packs past the last valid field carry no imaginary part
      const T* fa = src + (int64_t)q.x * nr + poff;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) ra[e] = fa[i];
      }
      if (q.y >= 0) {
        const T* fb = src + (int64_t)q.y * nr + poff;
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          const int i = threadIdx.x + e * kPlaneThreads;
          if (PL % kPlaneThreads == 0 || i < PL) rb[e] = fb[i];
        }
      } else {
#pragma unroll
        for (int e = 0; e < EL; ++e) rb[e] = T(1);
      }
      if (q.z >= 0) {
        const T* fc = src + (int64_t)q.z * nr + poff;
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          const int i = threadIdx.x + e * kPlaneThreads;
          if (PL % kPlaneThreads == 0 || i < PL) rc[e] = fc[i];
        }
      } else {
#pragma unroll
        for (int e = 0; e < EL; ++e) rc[e] = T(0);
      }
      if (q.z >= 0 && q.w >= 0) {
        const T* fd = src + (int64_t)q.w * nr + poff;
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          const int i = threadIdx.x + e * kPlaneThreads;
          if (PL % kPlaneThreads == 0 || i < PL) rd[e] = fd[i];
        }
      } else {
#pragma unroll
        for (int e = 0; e < EL; ++e) rd[e] = T(1);
      }
    };
    load(it0);
    for (int item = it0; item < it1; ++item) {
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) pl[i] = {ra[e] * rb[e], rc[e] * rd[e]};
      }
      __syncthreads();
      if (item + 1 < it1) load(item + 1);
      plane_fft<-1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
      const int i0 = item / npack;
      const int pack = item - i0 * npack;
      cplx<T>* o = dst + ((int64_t)pack * n0 + i0) * nds;
      for (int s = threadIdx.x; s < nd; s += blockDim.x) o[s] = pl[k12[s]];
      __syncthreads();
    }
  } else {
    const int item = xcd_item(total);
    if (item < 0) return;
    stage_twiddles<SN>(twl, tw1);
    const int i0 = item / npack;
    const int pack = item - i0 * npack;
    const int64_t poff = (int64_t)i0 * plane;
    int4 q = quads[pack];
    if (q.z >= limit) q.z = -1;  // packs past the last valid field carry no imaginary part
    const T* fa = src + (int64_t)q.x * nr + poff;
    const T* fb = q.y >= 0 ? src + (int64_t)q.y * nr + poff : nullptr;
    const T* fc = q.z >= 0 ? src + (int64_t)q.z * nr + poff : nullptr;
    const T* fd = q.w >= 0 ? src + (int64_t)q.w * nr + poff : nullptr;
    cplx<T>* o = dst + ((int64_t)pack * n0 + i0) * nds;
    if constexpr (SN > 0) {
      // every load of the item is issued before any is used (the density-stick
      // positions of the first kStickRegs rounds, then the four orbital planes),
      // so the item waits for one round trip instead of one per plane row
      constexpr int PL = SN * SN;
      constexpr int EL = (PL + kPlaneThreads - 1) / kPlaneThreads;
      constexpr int KS = stick_regs<SN>();
      int kp[KS];
#pragma unroll
      for (int e = 0; e < KS; ++e) {
        const int st = threadIdx.x + e * kPlaneThreads;
        kp[e] = st < nd ? k12[st] : -1;
      }
      // in two batches of plane rows, so the loads in flight fit the register
      // budget of three workgroups per CU
      constexpr int LB = (EL + 1) / 2;
#pragma unroll
      for (int e0 = 0; e0 < EL; e0 += LB) {
        T ra[LB], rb[LB], rc[LB], rd[LB];
#pragma unroll
        for (int e = 0; e < LB; ++e) {
          const int i = threadIdx.x + (e0 + e) * kPlaneThreads;
          if (e0 + e < EL && (PL % kPlaneThreads == 0 || i < PL)) {
            ra[e] = fa[i];
            rb[e] = fb ? fb[i] : T(1);
            rc[e] = fc ? fc[i] : T(0);
            rd[e] = fd ? fd[i] : T(1);
          }
        }
#pragma unroll
        for (int e = 0; e < LB; ++e) {
          const int i = threadIdx.x + (e0 + e) * kPlaneThreads;
          if (e0 + e < EL && (PL % kPlaneThreads == 0 || i < PL))
            pl[i] = {ra[e] * rb[e], rc[e] * rd[e]};
        }
      }
      __syncthreads();
      plane_fft<-1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
#pragma unroll
      for (int e = 0; e < KS; ++e)
        if (kp[e] >= 0) o[threadIdx.x + e * kPlaneThreads] = pl[kp[e]];
      for (int st = threadIdx.x + KS * kPlaneThreads; st < nd; st += blockDim.x)
        o[st] = pl[k12[st]];
    } else {
      for (int i = threadIdx.x; i < plane; i += blockDim.x) {
        T re = fb ? fa[i] * fb[i] : fa[i];
        T im = fc ? (fd ? fc[i] * fd[i] : fc[i]) : T(0);
        pl[i] = {re, im};
      }
      __syncthreads();
      plane_fft<-1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
      for (int st = threadIdx.x; st < nd; st += blockDim.x) o[st] = pl[k12[st]];
    }
  }
}

// ---------------------------------------------------------------- register-quad plane kernels
// For planes whose complex field does not fit in LDS (FP64 108 x 108): each
// line of SN points is held by a quad of lanes with SN / 4 points each
// (fft_quad_*), so the 2D FFT needs LDS only for the transpose between the row
// and the column transforms, restricted to the rows k1 that the stick set
// occupies.  rows[r] = (k1, first stick, R, 0): row r holds k2 = 0..R and
// SN - R..SN - 1 (sticks ordered by k1, then k2).  One (plane, pack) item per
// workgroup of quad_threads(SN) threads, quad qd = threadIdx / 4.
constexpr int quad_threads(int sn) { return (4 * sn + 63) / 64 * 64; }

// position of k2 within a stick row of half-width R, or -1
__device__ __forceinline__ int row_pos(int k2, int R, int sn) {
  return k2 <= R ? k2 : (k2 >= sn - R ? k2 - (sn - 2 * R - 1) : -1);
}

// rowof[k1] = stick row of k1, or -1 (callers synchronise before use)
template <int SN>
__device__ __forceinline__ void fill_rowof(int* rowof, const int4* __restrict__ rows, int nrow) {
  for (int k = threadIdx.x; k < SN; k += blockDim.x) rowof[k] = -1;
  __syncthreads();
  for (int r = threadIdx.x; r < nrow; r += blockDim.x) rowof[rows[r].x] = r;
}

// pair products -> density sticks: columns (along i1) straight from the
// orbital planes, the stick rows through LDS, then the rows (along i2)
template <int SN, typename T>
__global__ void __launch_bounds__(quad_threads(SN))
k_pairs_to_dsticks_q(const T* __restrict__ src, const int4* __restrict__ quads, int npack,
                     int limit, int n0, int nds, int nrow, const int4* __restrict__ rows,
                     cplx<T>* __restrict__ dst) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int M = SN / 4, TS = SN + 1, PL = SN * SN;
  cplx<T>* tr = reinterpret_cast<cplx<T>*>(smem_raw);  // [nrow][TS]
  int* rowof = reinterpret_cast<int*>(tr + nrow * TS);
  const int item = xcd_item(n0 * npack);
  if (item < 0) return;
  const int i0 = item / npack;
  const int pack = item - i0 * npack;
  fill_rowof<SN>(rowof, rows, nrow);
  __syncthreads();
  const int qd = threadIdx.x >> 2, e = threadIdx.x & 3, qb = quad_block(e);
  const int64_t nr = (int64_t)n0 * PL;
  int4 q = quads[pack];
  if (q.z >= limit) q.z = -1;  // packs past the last valid field carry no imaginary part
  if (qd < SN) {
    // column i2 = qd, points i1 = e M .. e M + M - 1; missing factors read the
    // first field again and are replaced by 1 (or the imaginary part by 0)
    const int64_t off = (int64_t)i0 * PL + (int64_t)(e * M) * SN + qd;
    const bool hb = q.y >= 0, hc = q.z >= 0, hd = q.z >= 0 && q.w >= 0;
    const T* fa = src + (int64_t)q.x * nr + off;
    const T* fb = src + (int64_t)(hb ? q.y : q.x) * nr + off;
    const T* fc = src + (int64_t)(hc ? q.z : q.x) * nr + off;
    const T* fd = src + (int64_t)(hd ? q.w : q.x) * nr + off;
    cplx<T> x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const T a = fa[m * SN], bb = fb[m * SN];
      x[m].x = hb ? a * bb : a;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const T c = fc[m * SN], d = fd[m * SN];
      x[m].y = hc ? (hd ? c * d : c) : T(0);
    }
    fft_quad_fwd_contig<SN>(x, e);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int r = rowof[4 * k + qb];
      if (r >= 0) tr[r * TS + qd] = x[k];
    }
  }
  __syncthreads();
  if (qd < nrow) {
    cplx<T> x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = tr[qd * TS + e * M + m];
    fft_quad_fwd_contig<SN>(x, e);
    const int4 rw = rows[qd];
    cplx<T>* o = dst + ((int64_t)pack * n0 + i0) * nds + rw.y;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int p = row_pos(4 * k + qb, rw.z, SN);
      if (p >= 0) o[p] = x[k];
    }
  }
}

// inverse 2D FFT of a pack of sticks: the stick rows (along k2) into LDS, then
// the columns (along k1); the lanes of column i2 hold points i1 = e M + m
template <int SN, typename T>
__device__ __forceinline__ void quad_plane_inverse(const cplx<T>* __restrict__ src, int nrow,
                                                   const int4* __restrict__ rows,
                                                   const int* rowof, cplx<T>* tr,
                                                   cplx<T> (&x)[SN / 4]) {
  constexpr int M = SN / 4, TS = SN + 1;
  const int qd = threadIdx.x >> 2, e = threadIdx.x & 3, qb = quad_block(e);
  if (qd < nrow) {
    const int4 rw = rows[qd];
    cplx<T> y[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int p = row_pos(4 * k + qb, rw.z, SN);
      y[k] = p >= 0 ? src[rw.y + p] : cplx<T>{T(0), T(0)};
    }
    fft_quad_inv_contig<SN>(y, e);
#pragma unroll
    for (int m = 0; m < M; ++m) tr[qd * TS + e * M + m] = y[m];
  }
  __syncthreads();
  if (qd < SN) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int r = rowof[4 * k + qb];
      x[k] = r >= 0 ? tr[r * TS + qd] : cplx<T>{T(0), T(0)};
    }
    fft_quad_inv_contig<SN>(x, e);
  }
}

// density sticks -> real fields (fields 2 pack and 2 pack + 1, [field][N_r])
template <int SN, typename T>
__global__ void __launch_bounds__(quad_threads(SN))
k_dsticks_to_fields_q(const cplx<T>* __restrict__ dst, int npack, int nfield, int n0, int nds,
                      int nrow, const int4* __restrict__ rows, T* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int M = SN / 4, TS = SN + 1, PL = SN * SN;
  cplx<T>* tr = reinterpret_cast<cplx<T>*>(smem_raw);
  int* rowof = reinterpret_cast<int*>(tr + nrow * TS);
  const int item = xcd_item(n0 * npack);
  if (item < 0) return;
  const int i0 = item / npack;
  const int pack = item - i0 * npack;
  fill_rowof<SN>(rowof, rows, nrow);
  __syncthreads();
  const int qd = threadIdx.x >> 2, e = threadIdx.x & 3;
  cplx<T> x[M];
  quad_plane_inverse<SN>(dst + ((int64_t)pack * n0 + i0) * nds, nrow, rows, rowof, tr, x);
  if (qd < SN) {
    const int64_t nr = (int64_t)n0 * PL;
    T* o1 = out + (int64_t)(2 * pack) * nr + (int64_t)i0 * PL + (int64_t)(e * M) * SN + qd;
    const bool has2 = 2 * pack + 1 < nfield;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      o1[m * SN] = x[m].x;
      if (has2) o1[nr + m * SN] = x[m].y;
    }
  }
}

// wave sticks -> real fields of the trial block, with the density response
// drho_b = sum_v phi_v out_bv accumulated in registers (each lane owns the same
// points for every pack); items (i0, group, b) as k_wsticks_to_fields
template <int SN, typename T>
__global__ void __launch_bounds__(quad_threads(SN))
k_wsticks_to_fields_q(const cplx<T>* __restrict__ wst, int npt, int per_trial, int n0, int nws,
                      int nrow, const int4* __restrict__ rows, T scale, T* __restrict__ out,
                      const T* __restrict__ phi, T* __restrict__ drho, int ngroup, int nbtot) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int M = SN / 4, TS = SN + 1, PL = SN * SN;
  cplx<T>* tr = reinterpret_cast<cplx<T>*>(smem_raw);
  int* rowof = reinterpret_cast<int*>(tr + nrow * TS);
  const int item = xcd_item(n0 * ngroup * nbtot);
  if (item < 0) return;
  const int i0 = item / (ngroup * nbtot);
  const int rem = item - i0 * ngroup * nbtot;
  const int grp = rem / nbtot, b = rem - grp * nbtot;
  const int per = (npt + ngroup - 1) / ngroup;
  const int j0 = grp * per, j1 = min(npt, j0 + per);
  fill_rowof<SN>(rowof, rows, nrow);
  __syncthreads();
  const int qd = threadIdx.x >> 2, e = threadIdx.x & 3;
  const int64_t nr = (int64_t)n0 * PL;
  // this lane's points: i1 = e M + m, i2 = qd
  const int64_t pofs = (int64_t)i0 * PL + (int64_t)(e * M) * SN + qd;
  T acc[M];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m] = T(0);
  for (int j = j0; j < j1; ++j) {
    cplx<T> x[M];
    quad_plane_inverse<SN>(wst + ((int64_t)(b * npt + j) * n0 + i0) * nws, nrow, rows, rowof, tr,
                           x);
    if (qd < SN) {
      const int v1 = 2 * j, v2 = 2 * j + 1;
      const bool has2 = v2 < per_trial;
      T* o1 = out + ((int64_t)b * per_trial + v1) * nr + pofs;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const T a = x[m].x * scale, c = x[m].y * scale;
        o1[m * SN] = a;
        if (has2) o1[nr + m * SN] = c;
        if (drho) {
          T d = phi[(int64_t)v1 * nr + pofs + m * SN] * a;
          if (has2) d += phi[(int64_t)v2 * nr + pofs + m * SN] * c;
          acc[m] += d;
        }
      }
    }
    __syncthreads();  // the next pack's rows overwrite the transpose buffer
  }
  if (drho && qd < SN) {
    T* d = drho + ((int64_t)grp * nbtot + b) * nr + pofs;
#pragma unroll
    for (int m = 0; m < M; ++m) d[m * SN] = acc[m];
  }
}

// real fields -> wave sticks: columns (along i1) from the two fields of a
// pack, the wave-stick rows through LDS, then the rows (along i2)
template <int SN, typename T>
__global__ void __launch_bounds__(quad_threads(SN))
k_fields_to_wsticks_q(const T* __restrict__ fields, int npt, int per_trial, int n0, int nws,
                      int nrow, const int4* __restrict__ rows, cplx<T>* __restrict__ wst,
                      int npack) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int M = SN / 4, TS = SN + 1, PL = SN * SN;
  cplx<T>* tr = reinterpret_cast<cplx<T>*>(smem_raw);
  int* rowof = reinterpret_cast<int*>(tr + nrow * TS);
  const int item = xcd_item(n0 * npack);
  if (item < 0) return;
  const int i0 = item / npack;
  const int pack = item - i0 * npack;
  fill_rowof<SN>(rowof, rows, nrow);
  __syncthreads();
  const int qd = threadIdx.x >> 2, e = threadIdx.x & 3, qb = quad_block(e);
  const int64_t nr = (int64_t)n0 * PL;
  if (qd < SN) {
    const int b = pack / npt, j = pack - b * npt;
    const int v1 = 2 * j, v2 = 2 * j + 1;
    const bool has2 = v2 < per_trial;
    const T* f1 = fields + ((int64_t)b * per_trial + v1) * nr + (int64_t)i0 * PL +
                  (int64_t)(e * M) * SN + qd;
    const T* f2 = has2 ? f1 + nr : f1;
    cplx<T> x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const T a = f1[m * SN], c = f2[m * SN];
      x[m] = {a, has2 ? c : T(0)};
    }
    fft_quad_fwd_contig<SN>(x, e);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int r = rowof[4 * k + qb];
      if (r >= 0) tr[r * TS + qd] = x[k];
    }
  }
  __syncthreads();
  if (qd < nrow) {
    cplx<T> x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = tr[qd * TS + e * M + m];
    fft_quad_fwd_contig<SN>(x, e);
    const int4 rw = rows[qd];
    cplx<T>* o = wst + ((int64_t)pack * n0 + i0) * nws + rw.y;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int p = row_pos(4 * k + qb, rw.z, SN);
      if (p >= 0) o[p] = x[k];
    }
  }
}

// ---------------------------------------------------------------- Poisson on density sticks
// forward FFT along i0, multiply by the kernel 4 pi/|G|^2 / N_r (v_g0/N_r at G = 0),
// inverse FFT along i0; in place.
template <int MB, int SN, typename T>
__global__ void __launch_bounds__(kStickThreads)
k_dstick_poisson(cplx<T>* __restrict__ dst, int n0, int nd, int nds, const T* __restrict__ kern,
                 FFTPlan P0, const cplx<T>* __restrict__ tw0, int ntile, int npack, int items) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tot = n0 * kStickTile;
  cplx<T>* twl = buf + tot;
  // items (pack, tile), tile fastest, `items` consecutive ones per workgroup in
  // XCD-contiguous ranges
  const int total = ntile * npack;
  const int grp = xcd_item((total + items - 1) / items);
  if (grp < 0) return;
  stage_twiddles<SN>(twl, tw0);
  const int it0 = grp * items, it1 = min(total, it0 + items);
  auto transform = [&](int tile, cplx<T>* base) {
    stick_fft<-1, SN, MB>(buf, P0, tw0, twl);
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
      const int k0 = i / kStickTile, l = i - k0 * kStickTile;
      const int s = tile * kStickTile + l;
      const T kv = (s < nd) ? kern[(int64_t)s * n0 + k0] : T(0);
      buf[i] = cscale(buf[i], kv);
    }
    __syncthreads();
    stick_fft<+1, SN, MB>(buf, P0, tw0, twl);
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
      const int i0 = i / kStickTile, l = i - i0 * kStickTile;
      const int s = tile * kStickTile + l;
      if (s < nd) base[(int64_t)i0 * nds + s] = buf[i];
    }
  };
  if constexpr (SN > 0) {
    // the next tile's sticks are loaded into registers while this one is transformed
    constexpr int EL = (SN * kStickTile + kStickThreads - 1) / kStickThreads;
    cplx<T> rv[EL];
    auto load = [&](int item) {
      const int pack = item / ntile, tile = item - pack * ntile;
      const cplx<T>* base = dst + (int64_t)pack * n0 * nds;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kStickThreads;
        const int i0 = i / kStickTile, l = i - i0 * kStickTile;
        const int s = tile * kStickTile + l;
        rv[e] = (i < tot && s < nd) ? base[(int64_t)i0 * nds + s] : cplx<T>{T(0), T(0)};
      }
    };
    load(it0);
    for (int item = it0; item < it1; ++item) {
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kStickThreads;
        if (i < tot) buf[i] = rv[e];
      }
      __syncthreads();
      if (item + 1 < it1) load(item + 1);
      const int pack = item / ntile, tile = item - pack * ntile;
      transform(tile, dst + (int64_t)pack * n0 * nds);
      __syncthreads();
    }
  } else {
    for (int item = it0; item < it1; ++item) {
      const int pack = item / ntile, tile = item - pack * ntile;
      cplx<T>* base = dst + (int64_t)pack * n0 * nds;
      for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int i0 = i / kStickTile, l = i - i0 * kStickTile;
        const int s = tile * kStickTile + l;
        buf[i] = (s < nd) ? base[(int64_t)i0 * nds + s] : cplx<T>{T(0), T(0)};
      }
      __syncthreads();
      transform(tile, base);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- density sticks -> real fields
// Items (plane i0, pack) in XCD-contiguous ranges, pack fastest.  The two real
// fields of pack p (fields 2p and 2p + 1) are written as planes of [field][N_r],
// or, with il, into the layout that interleaves groups of kTauIl fields point
// by point: field f at ((f / kTauIl) N_r + r) kTauIl + f % kTauIl (the packs of
// one group are neighbouring items, so their partial lines meet in one L2).
template <int MB1, int MB2, int SN, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_dsticks_to_fields(const cplx<T>* __restrict__ dst, int npack, int il, int nfield, int n0,
                    int n1, int n2, int nd, int nds,
                    const int* __restrict__ k12, FFTPlan P1, FFTPlan P2,
                    const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                    T* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  const int plane = n1 * n2;
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* twl = pl + plane;
  const int item = xcd_item(n0 * npack);
  if (item < 0) return;
  stage_twiddles<SN>(twl, tw1);
  const int i0 = item / npack;
  const int pack = item - i0 * npack;
  const int64_t nr = (int64_t)n0 * plane;
  const cplx<T>* src = dst + ((int64_t)pack * n0 + i0) * nds;
  // compile-time planes: the first kStickRegs rounds of stick loads are issued
  // before the plane is cleared
  constexpr int KR = (SN > 0) ? stick_regs<SN>() : 0;
  int kp[KR > 0 ? KR : 1];
  cplx<T> sv[KR > 0 ? KR : 1];
#pragma unroll
  for (int e = 0; e < KR; ++e) {
    const int st = threadIdx.x + e * kPlaneThreads;
    const bool in = st < nd;
    kp[e] = in ? k12[st] : -1;
    sv[e] = in ? src[st] : cplx<T>{T(0), T(0)};
  }
  for (int i = threadIdx.x; i < plane; i += blockDim.x) pl[i] = {T(0), T(0)};
  __syncthreads();
#pragma unroll
  for (int e = 0; e < KR; ++e)
    if (kp[e] >= 0) pl[kp[e]] = sv[e];
  for (int st = threadIdx.x + KR * kPlaneThreads; st < nd; st += blockDim.x)
    pl[k12[st]] = src[st];
  __syncthreads();
  plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
  const bool has2 = 2 * pack + 1 < nfield;
  if (il) {
    const int f = 2 * pack;
    T* o = out + (((int64_t)(f >> kTauIlShift) * nr + (int64_t)i0 * plane) << kTauIlShift) +
           (f & (kTauIl - 1));
    for (int i = threadIdx.x; i < plane; i += blockDim.x) {
      const cplx<T> z = pl[i];
      if (has2)
        *reinterpret_cast<cplx<T>*>(o + ((int64_t)i << kTauIlShift)) = z;
      else
        o[(int64_t)i << kTauIlShift] = z.x;
    }
  } else {
    T* o1 = out + (int64_t)(2 * pack) * nr + (int64_t)i0 * plane;
    T* o2 = o1 + nr;
    for (int i = threadIdx.x; i < plane; i += blockDim.x) {
      const cplx<T> z = pl[i];
      o1[i] = z.x;
      if (has2) o2[i] = z.y;
    }
  }
}

// Density sticks -> pair potentials in the 4-pair interleaved layout, for
// compile-time planes: item (plane i0, group q) transforms packs 2q and 2q + 1
// (the four fields of interleave group q) one after the other, keeps the first
// plane in registers and writes the four values of a point as one vector (16
// bytes in FP32), so every store of a wave covers whole lines; the second
// pack's first stick rounds load during the first transform.  A workgroup takes
// group_items() consecutive items; with more than one, the next item's first
// stick rounds load during the current item's second transform and stores.
// The stores carry the streaming hint: the pair potentials are read back only by
// the contraction, after every chunk (at 72^3 the stick Poisson of the chunks
// measured 3.19 -> 3.14 ms per apply with it, the apply 19.43 -> 19.35 ms).
template <int MB1, int MB2, int SN, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_dsticks_to_groups(const cplx<T>* __restrict__ dst, int npack, int nfield, int n0, int n1,
                    int n2, int nd, int nds, const int* __restrict__ k12, FFTPlan P1, FFTPlan P2,
                    const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                    T* __restrict__ out) {
  static_assert(SN > 0 && kTauIl == 4, "compile-time planes, 4-pair groups");
  typedef T v4 __attribute__((ext_vector_type(4)));
  extern __shared__ unsigned char smem_raw[];
  constexpr int PL = SN * SN;
  constexpr int EL = (PL + kPlaneThreads - 1) / kPlaneThreads;
  constexpr int KR = stick_regs<SN>();
  constexpr int NI = group_items<T>();
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* twl = pl + PL;
  if constexpr (NI == 1) {
    // (the one-item form on its own: written as the loop below with one
    // item it took 106 VGPRs instead of 79, two FP32 workgroups per CU
    // instead of three)
    const int ngrp = (npack + 1) / 2;
    const int item = xcd_item(n0 * ngrp);
    if (item < 0) return;
    stage_twiddles<SN>(twl, tw1);
    const int i0 = item / ngrp;
    const int q = item - i0 * ngrp;
    const int64_t nr = (int64_t)n0 * PL;
    const bool two = 2 * q + 1 < npack;
    int kp[KR];
    cplx<T> sv[KR];
    auto load = [&](int pack) {
      const cplx<T>* src = dst + ((int64_t)pack * n0 + i0) * nds;
#pragma unroll
      for (int e = 0; e < KR; ++e) {
        const int st = threadIdx.x + e * kPlaneThreads;
        sv[e] = kp[e] >= 0 ? src[st] : cplx<T>{T(0), T(0)};
      }
    };
    // fill the plane with pack `pack` (registers sv for the first rounds)
    auto fill = [&](int pack) {
      for (int i = threadIdx.x; i < PL; i += blockDim.x) pl[i] = {T(0), T(0)};
      __syncthreads();
#pragma unroll
      for (int e = 0; e < KR; ++e)
        if (kp[e] >= 0) pl[kp[e]] = sv[e];
      const cplx<T>* src = dst + ((int64_t)pack * n0 + i0) * nds;
      for (int st = threadIdx.x + KR * kPlaneThreads; st < nd; st += blockDim.x)
        pl[k12[st]] = src[st];
      __syncthreads();
    };
#pragma unroll
    for (int e = 0; e < KR; ++e) {
      const int st = threadIdx.x + e * kPlaneThreads;
      kp[e] = st < nd ? k12[st] : -1;
    }
    load(2 * q);
    fill(2 * q);
    if (two) load(2 * q + 1);
    plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
    cplx<T> keep[EL];
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int i = threadIdx.x + e * kPlaneThreads;
      if (PL % kPlaneThreads == 0 || i < PL) keep[e] = pl[i];
    }
    __syncthreads();
    if (two) {
      fill(2 * q + 1);
      plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
    }
    // group q holds fields 4q .. 4q + 3 (those below nfield exist)
    T* o = out + ((int64_t)q * nr + (int64_t)i0 * PL) * 4;
    const int f0 = 4 * q;
    const bool full = f0 + 3 < nfield;
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int i = threadIdx.x + e * kPlaneThreads;
      if (PL % kPlaneThreads == 0 || i < PL) {
        const cplx<T> b = two ? pl[i] : cplx<T>{T(0), T(0)};
        if (full) {
          __builtin_nontemporal_store(v4{keep[e].x, keep[e].y, b.x, b.y},
                                       reinterpret_cast<v4*>(o + 4 * (int64_t)i));
        } else {
          o[4 * (int64_t)i] = keep[e].x;
          if (f0 + 1 < nfield) o[4 * (int64_t)i + 1] = keep[e].y;
          if (f0 + 2 < nfield) o[4 * (int64_t)i + 2] = b.x;
        }
      }
    }
  } else {
    const int ngrp = (npack + 1) / 2;
    const int total = n0 * ngrp;
    const int wg = xcd_item((total + NI - 1) / NI);
    if (wg < 0) return;
    stage_twiddles<SN>(twl, tw1);
    const int it0 = wg * NI, it1 = min(total, it0 + NI);
    const int64_t nr = (int64_t)n0 * PL;
    int kp[KR];
    cplx<T> sv[KR];
    auto load = [&](int pack, int i0) {
      const cplx<T>* src = dst + ((int64_t)pack * n0 + i0) * nds;
#pragma unroll
      for (int e = 0; e < KR; ++e) {
        const int st = threadIdx.x + e * kPlaneThreads;
        sv[e] = kp[e] >= 0 ? src[st] : cplx<T>{T(0), T(0)};
      }
    };
    // fill the plane with pack `pack` (registers sv for the first rounds)
    auto fill = [&](int pack, int i0) {
      for (int i = threadIdx.x; i < PL; i += blockDim.x) pl[i] = {T(0), T(0)};
      __syncthreads();
#pragma unroll
      for (int e = 0; e < KR; ++e)
        if (kp[e] >= 0) pl[kp[e]] = sv[e];
      const cplx<T>* src = dst + ((int64_t)pack * n0 + i0) * nds;
      for (int st = threadIdx.x + KR * kPlaneThreads; st < nd; st += blockDim.x)
        pl[k12[st]] = src[st];
      __syncthreads();
    };
#pragma unroll
    for (int e = 0; e < KR; ++e) {
      const int st = threadIdx.x + e * kPlaneThreads;
      kp[e] = st < nd ? k12[st] : -1;
    }
    load(2 * (it0 % ngrp), it0 / ngrp);
    for (int item = it0; item < it1; ++item) {
      const bool next = item + 1 < it1;
      const int i0 = item / ngrp;
      const int q = item - i0 * ngrp;
      const bool two = 2 * q + 1 < npack;
      fill(2 * q, i0);
      if (two) load(2 * q + 1, i0);
      plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
      cplx<T> keep[EL];
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) keep[e] = pl[i];
      }
      __syncthreads();
      if (two) fill(2 * q + 1, i0);
      if (next) load(2 * ((item + 1) % ngrp), (item + 1) / ngrp);
      if (two) plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
      // group q holds fields 4q .. 4q + 3 (those below nfield exist)
      T* o = out + ((int64_t)q * nr + (int64_t)i0 * PL) * 4;
      const int f0 = 4 * q;
      const bool full = f0 + 3 < nfield;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) {
          const cplx<T> b = two ? pl[i] : cplx<T>{T(0), T(0)};
          if (full) {
            __builtin_nontemporal_store(v4{keep[e].x, keep[e].y, b.x, b.y},
                                         reinterpret_cast<v4*>(o + 4 * (int64_t)i));
          } else {
            o[4 * (int64_t)i] = keep[e].x;
            if (f0 + 1 < nfield) o[4 * (int64_t)i + 1] = keep[e].y;
            if (f0 + 2 < nfield) o[4 * (int64_t)i + 2] = b.x;
          }
        }
      }
      // (the next item's fill clears the plane these stores read)
      if (next) __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- K2d: inverse pass + contraction
// Pack p = j (nocc / 2) + k of dst holds the Poisson-solved products a_bv' phi_v
// and a_bv' phi_v+1 (v' = r0 + j, v = 2k) on density sticks.  The workgroup of
// item (plane i0, k) transforms the packs of every row j back to the plane and
// sums phi_v'(r) W_v'v(r) for v and v + 1 in registers, then applies
// R_bv -= alpha sum once per plane (no W fields in HBM).
template <int MB1, int MB2, int SN, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_k2d_inverse(const cplx<T>* __restrict__ dst, int nrows, int r0, int nocc, int n0, int n1,
              int n2, int nd, int nds, const int* __restrict__ k12, FFTPlan P1, FFTPlan P2,
              const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
              const T* __restrict__ phi, T alpha, T* __restrict__ R) {
  if constexpr (SN == 72) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int PL = SN * SN;
    constexpr int EL = (PL + kPlaneThreads - 1) / kPlaneThreads;
    constexpr int KR = kStickRegs;
    cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* twl = pl + PL;
    const int hp = nocc / 2;
    const int item = xcd_item(n0 * hp);
    if (item < 0) return;
    stage_twiddles<SN>(twl, tw1);
    const int i0 = item / hp;
    const int k = item - i0 * hp;
    const int64_t nr = (int64_t)n0 * PL;
    const int64_t poff = (int64_t)i0 * PL;
    // stick positions are the same for every pack: taken once
    int kp[KR];
#pragma unroll
    for (int e = 0; e < KR; ++e) {
      const int st = threadIdx.x + e * kPlaneThreads;
      kp[e] = st < nd ? k12[st] : -1;
    }
    cplx<T> sv[KR];
    auto load_sticks = [&](int j) {
      const cplx<T>* src = dst + ((int64_t)(j * hp + k) * n0 + i0) * nds;
#pragma unroll
      for (int e = 0; e < KR; ++e)
        sv[e] = kp[e] >= 0 ? src[threadIdx.x + e * kPlaneThreads] : cplx<T>{T(0), T(0)};
    };
    T acc1[EL], acc2[EL];
#pragma unroll
    for (int e = 0; e < EL; ++e) acc1[e] = acc2[e] = T(0);
    load_sticks(0);
    for (int j = 0; j < nrows; ++j) {
      for (int i = threadIdx.x; i < PL; i += kPlaneThreads) pl[i] = {T(0), T(0)};
      __syncthreads();
#pragma unroll
      for (int e = 0; e < KR; ++e)
        if (kp[e] >= 0) pl[kp[e]] = sv[e];
      {
        const cplx<T>* src = dst + ((int64_t)(j * hp + k) * n0 + i0) * nds;
        for (int st = threadIdx.x + KR * kPlaneThreads; st < nd; st += kPlaneThreads)
          pl[k12[st]] = src[st];
      }
      __syncthreads();
      if (j + 1 < nrows) load_sticks(j + 1);
      T f[EL];
      const T* ph = phi + (int64_t)(r0 + j) * nr + poff;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        f[e] = (PL % kPlaneThreads == 0 || i < PL) ? ph[i] : T(0);
      }
      plane_fft<+1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) {
          const cplx<T> z = pl[i];
          acc1[e] += f[e] * z.x;
          acc2[e] += f[e] * z.y;
        }
      }
      __syncthreads();
    }
    T* o1 = R + (int64_t)(2 * k) * nr + poff;
    T* o2 = o1 + nr;
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int i = threadIdx.x + e * kPlaneThreads;
      if (PL % kPlaneThreads == 0 || i < PL) {
        o1[i] -= alpha * acc1[e];
        o2[i] -= alpha * acc2[e];
      }
    }
  }
}

// ---------------------------------------------------------------- real fields -> wave sticks
// Items (plane i0, pack) in XCD-contiguous ranges, `items` consecutive items per
// workgroup; on compile-time planes the next item's two fields are loaded into
// registers while the current plane is transformed.
template <int MB1, int MB2, int SN, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_fields_to_wsticks(const T* __restrict__ fields, int npt, int per_trial, int items, int n0,
                    int n1, int n2, int nw, int nws, const int* __restrict__ k12, FFTPlan P1,
                    FFTPlan P2, const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                    cplx<T>* __restrict__ wst, int npack) {
  extern __shared__ unsigned char smem_raw[];
  const int plane = n1 * n2;
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* twl = pl + plane;
  const int64_t nr = (int64_t)n0 * plane;
  const int total = n0 * npack;
  const int grp = xcd_item((total + items - 1) / items);
  if (grp < 0) return;
  stage_twiddles<SN>(twl, tw1);
  const int it0 = grp * items, it1 = min(total, it0 + items);
  // item -> the pack's two fields at plane i0 (f2 = nullptr for an odd last orbital)
  auto fields_of = [&](int item, const T*& f1, const T*& f2, int& i0, int& pack) {
    i0 = item / npack;
    pack = item - i0 * npack;
    const int b = pack / npt, j = pack - b * npt;
    const int v1 = 2 * j, v2 = 2 * j + 1;
    f1 = fields + ((int64_t)b * per_trial + v1) * nr + (int64_t)i0 * plane;
    f2 = (v2 < per_trial) ? f1 + nr : nullptr;
  };
  auto finish = [&](int i0, int pack) {
    plane_fft<-1, SN, MB1, MB2>(pl, P1, P2, n1, n2, tw1, tw2, twl);
    cplx<T>* o = wst + ((int64_t)pack * n0 + i0) * nws;
    for (int st = threadIdx.x; st < nw; st += blockDim.x) o[st] = pl[k12[st]];
  };
  if constexpr (SN > 0) {
    constexpr int PL = SN * SN;
    constexpr int EL = (PL + kPlaneThreads - 1) / kPlaneThreads;
    T r1[EL], r2[EL];
    auto load = [&](int item) {
      const T *f1, *f2;
      int i0, pack;
      fields_of(item, f1, f2, i0, pack);
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) {
          r1[e] = f1[i];
          r2[e] = f2 ? f2[i] : T(0);
        }
      }
    };
    load(it0);
    for (int item = it0; item < it1; ++item) {
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int i = threadIdx.x + e * kPlaneThreads;
        if (PL % kPlaneThreads == 0 || i < PL) pl[i] = {r1[e], r2[e]};
      }
      __syncthreads();
      if (item + 1 < it1) load(item + 1);
      const int i0 = item / npack;
      finish(i0, item - i0 * npack);
      __syncthreads();
    }
  } else {
    for (int item = it0; item < it1; ++item) {
      const T *f1, *f2;
      int i0, pack;
      fields_of(item, f1, f2, i0, pack);
      for (int i = threadIdx.x; i < plane; i += blockDim.x) pl[i] = {f1[i], f2 ? f2[i] : T(0)};
      __syncthreads();
      finish(i0, pack);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- wave sticks: forward along i0
template <int MB, int SN, typename T>
__global__ void __launch_bounds__(kStickThreads)
k_wsticks_forward(cplx<T>* __restrict__ wst, int n0, int nw, int nws, FFTPlan P0,
                  const cplx<T>* __restrict__ tw0) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tile = blockIdx.x;
  const int pack = blockIdx.y;
  cplx<T>* base = wst + (int64_t)pack * n0 * nws;
  const int tot = n0 * kStickTile;
  cplx<T>* twl = buf + tot;
  stage_twiddles<SN>(twl, tw0);
  for (int i = threadIdx.x; i < tot; i += blockDim.x) {
    const int i0 = i / kStickTile, l = i - i0 * kStickTile;
    const int s = tile * kStickTile + l;
    buf[i] = (s < nw) ? base[(int64_t)i0 * nws + s] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  stick_fft<-1, SN, MB>(buf, P0, tw0, twl);
  for (int i = threadIdx.x; i < tot; i += blockDim.x) {
    const int k0 = i / kStickTile, l = i - k0 * kStickTile;
    const int s = tile * kStickTile + l;
    if (s < nw) base[(int64_t)k0 * nws + s] = buf[i];
  }
}

// ---------------------------------------------------------------- unpack to half-sphere coefficients
// F1(m) = (Z(m) + conj Z(-m)) / 2, F2(m) = (Z(m) - conj Z(-m)) / (2i), times scale.
template <typename T>
__global__ void k_extract_sphere(const cplx<T>* __restrict__ wst, int npt, int per_trial,
                                 int n0, int nws, int npw, const int2* __restrict__ pos, T scale,
                                 T* __restrict__ coef) {
  const int pack = blockIdx.y;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= npw) return;
  const int b = pack / npt, j = pack - b * npt;
  const int v1 = 2 * j, v2 = 2 * j + 1;
  const cplx<T>* base = wst + (int64_t)pack * n0 * nws;
  const int2 ps = pos[h];
  const cplx<T> zp = base[ps.x], zm = base[ps.y];
  const T hs = T(0.5) * scale;
  T* c1 = coef + (((int64_t)b * per_trial + v1) * npw + h) * 2;
  c1[0] = (zp.x + zm.x) * hs;
  c1[1] = (zp.y - zm.y) * hs;
  if (v2 < per_trial) {
    T* c2 = c1 + (int64_t)npw * 2;
    c2[0] = (zp.y + zm.y) * hs;
    c2[1] = (zm.x - zp.x) * hs;
  }
}

// ---------------------------------------------------------------- exchange + response contraction
// R[b][v](r) = c_K phi_v(r) (v_H,b(r) + f_xc(r) drho_b(r)) - alpha sum_v' tau_vv'(r) a~[b][v'](r)
// Tile: 64 points x 16 occupied rows x 16 trials; loop over v' in chunks of 4
// staged in LDS.  Each thread owns one point and 4 rows (64 accumulators).
constexpr int kCtPts = 64, kCtV = 16, kCtB = 16, kCtVp = 4;

template <typename T>
__global__ void __launch_bounds__(256)
k_contract(int nb, int nocc, int64_t nr, int ntile, int nvb, const T* __restrict__ phi,
           const T* __restrict__ at, const T* __restrict__ tau, const int* __restrict__ pidx,
           const T* __restrict__ vh, const T* __restrict__ drho, const T* __restrict__ fxc,
           T ck, T alpha, int k1e, int k1d, T* __restrict__ R) {
  __shared__ T s_tau[kCtV][kCtVp][kCtPts];
  __shared__ T s_at[kCtB][kCtVp][kCtPts];
  // XCD-aware order: consecutive dispatch slots on one XCD are the v-blocks of
  // one point tile, so the trial fields of that tile are shared through L2.
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int vb = slot % nvb;
  const int tile = (slot / nvb) * 8 + xcd;
  if (tile >= ntile) return;
  const int64_t r0 = (int64_t)tile * kCtPts;
  const int tid = threadIdx.x;
  const int pt = tid & (kCtPts - 1);
  const int vs = tid >> 6;  // 0..3
  const int64_t r = r0 + pt;
  const bool rin = r < nr;
  for (int b0 = 0; b0 < nb; b0 += kCtB) {
    T acc[4][kCtB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bb = 0; bb < kCtB; ++bb) acc[a][bb] = T(0);
    if (k1d) {
      for (int vp0 = 0; vp0 < nocc; vp0 += kCtVp) {
        // stage tau[v-block][vp chunk][pts] and at[b chunk][vp chunk][pts]
        for (int e = tid; e < kCtV * kCtVp * kCtPts; e += 256) {
          const int p = e & (kCtPts - 1), q = e >> 6;
          const int vv = q / kCtVp, vp = q - vv * kCtVp;
          const int v = vb * kCtV + vv, vpa = vp0 + vp;
          const int64_t rr = r0 + p;
          T val = T(0);
          if (v < nocc && vpa < nocc && rr < nr) val = tau[(int64_t)pidx[v * nocc + vpa] * nr + rr];
          s_tau[vv][vp][p] = val;
        }
        for (int e = tid; e < kCtB * kCtVp * kCtPts; e += 256) {
          const int p = e & (kCtPts - 1), q = e >> 6;
          const int bb = q / kCtVp, vp = q - bb * kCtVp;
          const int b = b0 + bb, vpa = vp0 + vp;
          const int64_t rr = r0 + p;
          T val = T(0);
          if (b < nb && vpa < nocc && rr < nr) val = at[((int64_t)b * nocc + vpa) * nr + rr];
          s_at[bb][vp][p] = val;
        }
        __syncthreads();
#pragma unroll
        for (int vp = 0; vp < kCtVp; ++vp) {
          T t[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) t[a] = s_tau[vs * 4 + a][vp][pt];
#pragma unroll
          for (int bb = 0; bb < kCtB; ++bb) {
            const T x = s_at[bb][vp][pt];
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a][bb] += t[a] * x;
          }
        }
        __syncthreads();
      }
    }
    if (rin) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int v = vb * kCtV + vs * 4 + a;
        if (v >= nocc) continue;
        const T ph = phi[(int64_t)v * nr + r];
        for (int bb = 0; bb < kCtB; ++bb) {
          const int b = b0 + bb;
          if (b >= nb) break;
          T val = -alpha * acc[a][bb];
          if (k1e) {
            const T d = drho[(int64_t)b * nr + r];
            val += ck * ph * (vh[(int64_t)b * nr + r] + fxc[r] * d);
          }
          R[((int64_t)b * nocc + v) * nr + r] = val;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- small elementwise kernels
template <typename T>
__global__ void k_dterm_combine(int nb, int nocc, int nc, const T* __restrict__ S,
                                const T* __restrict__ Q, const double* __restrict__ eo,
                                const double* __restrict__ ec, int with_d, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * nocc * nc;
  if (i >= tot) return;
  const int c = (int)(i % nc);
  const int v = (int)((i / nc) % nocc);
  T val = Q[i];
  if (with_d) val += (T)(ec[c] - eo[v]) * S[i];
  out[i] = val;
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ in, Tout* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (Tout)in[i];
}

// Clears n elements (a kernel rather than a memset node, so callers may capture it in a graph).
template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = (T)0;
}

__global__ void k_transition_out(int nb, int nocc, int nc, const void* __restrict__ Q, int qf,
                                 const double* __restrict__ X, const double* __restrict__ eo,
                                 const double* __restrict__ ec, int with_d,
                                 double* __restrict__ T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * nocc * nc;
  if (i >= tot) return;
  const int c = (int)(i % nc);
  const int v = (int)((i / nc) % nocc);
  double q = qf ? (double)reinterpret_cast<const float*>(Q)[i]
                : reinterpret_cast<const double*>(Q)[i];
  if (with_d) q += (ec[c] - eo[v]) * X[i];
  T[i] = q;
}

template <typename F>
void set_lds(F* func, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(func),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void check_lds(size_t bytes) {
  WTD_REQUIRE(bytes <= 160 * 1024, WTD_ERR_SHAPE,
              "grid plane does not fit in 160 KB of LDS for this precision");
}

}  // namespace

// ============================================================================ launchers
// Grid sizes with compile-time FFT plans (the benchmark's 72 and 108 and the
// batch's 48, 60 and 96); other sizes use the runtime plans.
int static_size(int n) {
  return (n == 48 || n == 60 || n == 72 || n == 96 || n == 108) ? n : 0;
}
int plane_static(const Geometry& g) { return g.n1 == g.n2 ? static_size(g.n1) : 0; }

#define WTD_STICK_CASE(N, K, T, grid, lds0, stream, ...)                                     \
  case N: {                                                                                 \
    const size_t l_ = (lds0) + N * sizeof(cplx<T>);                                         \
    set_lds((K<1, N, T>), l_);                                                              \
    hipLaunchKernelGGL((K<1, N, T>), grid, dim3(kStickThreads), l_, stream, __VA_ARGS__);   \
  } break;

// Launch a stick kernel K<MB, SN, T> with the right static size or radix bound.
#define WTD_STICK_LAUNCH(K, T, grid, lds0, stream, ...)                                     \
  do {                                                                                      \
    switch (static_size(g.n0)) {                                                            \
      WTD_STICK_CASE(48, K, T, grid, lds0, stream, __VA_ARGS__)                             \
      WTD_STICK_CASE(60, K, T, grid, lds0, stream, __VA_ARGS__)                             \
      WTD_STICK_CASE(72, K, T, grid, lds0, stream, __VA_ARGS__)                             \
      WTD_STICK_CASE(96, K, T, grid, lds0, stream, __VA_ARGS__)                             \
      WTD_STICK_CASE(108, K, T, grid, lds0, stream, __VA_ARGS__)                            \
      default: {                                                                            \
        const int mb_ = pick_maxb(kStickTile, g.plan0, kStickThreads);                      \
        WTD_MAXB_DISPATCH(mb_, {                                                            \
          set_lds((K<MB, 0, T>), (lds0));                                                   \
          hipLaunchKernelGGL((K<MB, 0, T>), grid, dim3(kStickThreads), (lds0), stream,      \
                             __VA_ARGS__);                                                  \
        });                                                                                 \
      }                                                                                     \
    }                                                                                       \
    WTD_HIP(hipGetLastError());                                                             \
  } while (0)

#define WTD_PLANE_CASE(N, K, T, grid, lds0, stream, ...)                                     \
  case N: {                                                                                 \
    const size_t l_ = (lds0) + N * sizeof(cplx<T>);                                         \
    check_lds(l_);                                                                          \
    set_lds((K<1, 1, N, T>), l_);                                                           \
    hipLaunchKernelGGL((K<1, 1, N, T>), grid, dim3(kPlaneThreads), l_, stream, __VA_ARGS__); \
  } break;

// Launch a plane kernel K<MB1, MB2, SN, T> with the compile-time plan of size
// SN_ (0: runtime plans).
#define WTD_PLANE_LAUNCH_SN(SN_, K, T, grid, lds0, stream, ...)                              \
  do {                                                                                       \
    switch (SN_) {                                                                           \
      WTD_PLANE_CASE(48, K, T, grid, lds0, stream, __VA_ARGS__)                              \
      WTD_PLANE_CASE(60, K, T, grid, lds0, stream, __VA_ARGS__)                              \
      WTD_PLANE_CASE(72, K, T, grid, lds0, stream, __VA_ARGS__)                              \
      WTD_PLANE_CASE(96, K, T, grid, lds0, stream, __VA_ARGS__)                              \
      WTD_PLANE_CASE(108, K, T, grid, lds0, stream, __VA_ARGS__)                             \
      default: {                                                                             \
        check_lds(lds0);                                                                     \
        const int mb1_ = pick_maxb(g.n2, g.plan1, kPlaneThreads);                            \
        const int mb2_ = pick_maxb(g.n1, g.plan2, kPlaneThreads);                            \
        WTD_MAXB_DISPATCH(mb1_, {                                                            \
          constexpr int M1 = MB;                                                             \
          WTD_MAXB_DISPATCH(mb2_, {                                                          \
            constexpr int M2 = MB;                                                           \
            set_lds((K<M1, M2, 0, T>), (lds0));                                              \
            hipLaunchKernelGGL((K<M1, M2, 0, T>), grid, dim3(kPlaneThreads), (lds0), stream, \
                               __VA_ARGS__);                                                 \
          });                                                                                \
        });                                                                                  \
      }                                                                                      \
    }                                                                                        \
    WTD_HIP(hipGetLastError());                                                              \
  } while (0)

#define WTD_PLANE_LAUNCH(K, T, grid, lds0, stream, ...) \
  WTD_PLANE_LAUNCH_SN(plane_static(g), K, T, grid, lds0, stream, __VA_ARGS__)

// the same for kernels that exist for compile-time planes only
#define WTD_PLANE_LAUNCH_STATIC(K, T, grid, lds0, stream, ...)                           \
  do {                                                                                  \
    switch (plane_static(g)) {                                                          \
      WTD_PLANE_CASE(48, K, T, grid, lds0, stream, __VA_ARGS__)                         \
      WTD_PLANE_CASE(60, K, T, grid, lds0, stream, __VA_ARGS__)                         \
      WTD_PLANE_CASE(72, K, T, grid, lds0, stream, __VA_ARGS__)                         \
      WTD_PLANE_CASE(96, K, T, grid, lds0, stream, __VA_ARGS__)                         \
      WTD_PLANE_CASE(108, K, T, grid, lds0, stream, __VA_ARGS__)                        \
      default:                                                                          \
        throw StatusError{WTD_ERR_SHAPE, "plane size without a compile-time FFT plan"}; \
    }                                                                                   \
    WTD_HIP(hipGetLastError());                                                         \
  } while (0)

// static size for the wave-stick plane kernels, which keep the wave sticks of
// an item in wave_stick_regs<SN>() registers per thread (runtime plans where
// the sphere has more sticks than that holds)
int plane_static_wave(const Geometry& g) {
  const int sn = plane_static(g);
  const int ws = sn >= 96 ? 3 : 2;
  return (sn > 0 && g.nw <= ws * kPlaneThreads) ? sn : 0;
}

// the register-quad plane kernels: square planes of 24, 48, 72, 96 or 108
// points whose stick sets are row-regular, taken where the complex plane and
// its twiddles do not fit in LDS (FP64 108 x 108) or, with force, everywhere
int quad_plane_size(const Geometry& g, size_t elem, bool force) {
  const int n = g.n1 == g.n2 ? g.n1 : 0;
  if (!(n == 24 || n == 48 || n == 72 || n == 96 || n == 108) || g.ndrow <= 0 || g.nwrow <= 0)
    return 0;
  const bool fits = (size_t)(n * n + n) * 2 * elem <= 160 * 1024;
  return (force || !fits) ? n : 0;
}

#define WTD_QUAD_LAUNCH(K, T, nrow, items, stream, ...)                                      \
  do {                                                                                       \
    switch (g.quad_sn) {                                                                     \
      WTD_QUAD_CASE(24, K, T, nrow, items, stream, __VA_ARGS__)                              \
      WTD_QUAD_CASE(48, K, T, nrow, items, stream, __VA_ARGS__)                              \
      WTD_QUAD_CASE(72, K, T, nrow, items, stream, __VA_ARGS__)                              \
      WTD_QUAD_CASE(96, K, T, nrow, items, stream, __VA_ARGS__)                              \
      WTD_QUAD_CASE(108, K, T, nrow, items, stream, __VA_ARGS__)                             \
      default:                                                                               \
        throw StatusError{WTD_ERR_SHAPE, "no register-quad plane kernel for this grid"};    \
    }                                                                                        \
    WTD_HIP(hipGetLastError());                                                              \
  } while (0)
#define WTD_QUAD_CASE(N, K, T, nrow, items, stream, ...)                                     \
  case N: {                                                                                  \
    const size_t l_ = (size_t)(nrow) * (N + 1) * sizeof(cplx<T>) + N * sizeof(int);          \
    check_lds(l_);                                                                           \
    set_lds((K<N, T>), l_);                                                                  \
    hipLaunchKernelGGL((K<N, T>), dim3((unsigned)(((items) + 7) / 8 * 8)),                   \
                       dim3(quad_threads(N)), l_, stream, __VA_ARGS__);                      \
  } break;

template <typename T>
void launch_sphere_to_wsticks(const Geometry& g, const T* coef, int nfield, int npw, int nb,
                              int per_trial, cplx<T>* wst, hipStream_t s) {
  (void)nfield;
  const int npt = (per_trial + 1) / 2;
  dim3 grid(g.nwtile, nb * npt);
  const size_t lds = (size_t)g.n0 * kStickTile * sizeof(cplx<T>);
  WTD_STICK_LAUNCH(k_sphere_to_wsticks, T, grid, lds, s, coef, per_trial, npt, npw, g.n0, g.nw,
                   g.nws, g.wtile_off, g.wtile_ent, g.plan0, static_cast<const cplx<T>*>(g.tw0), wst);
}

template <typename T>
void launch_wsticks_to_fields(const Geometry& g, const cplx<T>* wst, int nb, int per_trial,
                              int nfield_per_trial, T scale, T* out, const T* phi, T* drho,
                              hipStream_t s, T* part, int ngroup) {
  (void)nfield_per_trial;
  const int npt = (per_trial + 1) / 2;
  if (!drho || !part) ngroup = 1;
  ngroup = std::max(1, std::min(ngroup, npt));
  if (g.quad_sn > 0) {
    T* dt = (ngroup > 1) ? part : drho;
    WTD_QUAD_LAUNCH(k_wsticks_to_fields_q, T, g.nwrow, g.n0 * nb * ngroup, s, wst, npt,
                    per_trial, g.n0, g.nws, g.nwrow, g.wrows, scale, out, phi, dt, ngroup, nb);
  } else {
  dim3 grid((unsigned)((g.n0 * nb * ngroup + 7) / 8 * 8));
  const int sn = plane_static_wave(g);
  // compile-time plans accumulate the density in registers, runtime plans in LDS
  const size_t lds = (size_t)g.plane * (sizeof(cplx<T>) + (drho && sn == 0 ? sizeof(T) : 0));
  T* dtarget = (ngroup > 1) ? part : drho;
  WTD_PLANE_LAUNCH_SN(sn, k_wsticks_to_fields, T, grid, lds, s, wst, npt,
                      per_trial, g.n0, g.n1, g.n2,
                   g.nw, g.nws, g.wst_k12, g.plan1w, g.plan2, static_cast<const cplx<T>*>(g.tw1),
                   static_cast<const cplx<T>*>(g.tw2), scale, out, phi, dtarget, ngroup, nb);
  }
  if (ngroup > 1) {
    const int64_t n = (int64_t)nb * g.nr;
    hipLaunchKernelGGL(k_sum_groups<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                       ngroup, n, drho);
    WTD_HIP(hipGetLastError());
  }
}

template <typename T>
void launch_pairs_to_dsticks(const Geometry& g, const T* src, const int4* quads, int npack,
                             int limit, cplx<T>* dst, hipStream_t s) {
  if (g.quad_sn > 0) {
    WTD_QUAD_LAUNCH(k_pairs_to_dsticks_q, T, g.ndrow, g.n0 * npack, s, src, quads, npack, limit,
                    g.n0, g.nds, g.ndrow, g.drows, dst);
    return;
  }
  const int ps = plane_static(g);
  const int per_wg = (ps > 0 && ps * ps <= 72 * 72 && sizeof(T) == 8) ? kPairItems : 1;
  const int ngrp = (g.n0 * npack + per_wg - 1) / per_wg;
  dim3 grid((unsigned)((ngrp + 7) / 8 * 8));
  const size_t lds = (size_t)g.plane * sizeof(cplx<T>);
  WTD_PLANE_LAUNCH(k_pairs_to_dsticks, T, grid, lds, s, src, quads, npack, limit, g.n0, g.n1,
                   g.n2, g.nd, g.nds, g.dst_k12, g.plan1d, g.plan2, static_cast<const cplx<T>*>(g.tw1),
                   static_cast<const cplx<T>*>(g.tw2), dst);
}

template <typename T>
void launch_dstick_poisson(const Geometry& g, cplx<T>* dst, int npack, hipStream_t s) {
  const int ntile = (g.nd + kStickTile - 1) / kStickTile;
  // several tiles per workgroup, the next one's sticks prefetched into
  // registers (FP64: two; 1 and 4 measured 6 and 1 % slower at 72^3)
  const int items = static_size(g.n0) ? (sizeof(T) == 4 ? kPairItems : 2) : 1;
  const int ngrp = (ntile * npack + items - 1) / items;
  dim3 grid((unsigned)((ngrp + 7) / 8 * 8));
  const size_t lds = (size_t)g.n0 * kStickTile * sizeof(cplx<T>);
  WTD_STICK_LAUNCH(k_dstick_poisson, T, grid, lds, s, dst, g.n0, g.nd, g.nds,
                   static_cast<const T*>(g.dkern), g.plan0, static_cast<const cplx<T>*>(g.tw0),
                   ntile, npack, items);
}

template <typename T>
void launch_dsticks_to_fields(const Geometry& g, const cplx<T>* dst, int npack, int nfield,
                              T* out, hipStream_t s, bool il) {
  if (g.quad_sn > 0 && !il) {
    WTD_QUAD_LAUNCH(k_dsticks_to_fields_q, T, g.ndrow, g.n0 * npack, s, dst, npack, nfield, g.n0,
                    g.nds, g.ndrow, g.drows, out);
    return;
  }
  // (not on 96 x 96 planes: the kept plane takes the group kernel above 128
  // VGPRs, one workgroup per CU where the LDS holds two)
  if (il && plane_static(g) > 0 && plane_static(g) != 96) {
    const int ngrp = (npack + 1) / 2;
    const int wgs = (g.n0 * ngrp + group_items<T>() - 1) / group_items<T>();
    dim3 grid((unsigned)((wgs + 7) / 8 * 8));
    const size_t lds = (size_t)g.plane * sizeof(cplx<T>);
    WTD_PLANE_LAUNCH_STATIC(k_dsticks_to_groups, T, grid, lds, s, dst, npack, nfield, g.n0, g.n1,
                            g.n2, g.nd, g.nds, g.dst_k12, g.plan1d, g.plan2,
                            static_cast<const cplx<T>*>(g.tw1), static_cast<const cplx<T>*>(g.tw2),
                            out);
    return;
  }
  dim3 grid((unsigned)((g.n0 * npack + 7) / 8 * 8));
  const size_t lds = (size_t)g.plane * sizeof(cplx<T>);
  WTD_PLANE_LAUNCH(k_dsticks_to_fields, T, grid, lds, s, dst, npack, il ? 1 : 0, nfield, g.n0,
                   g.n1, g.n2, g.nd, g.nds, g.dst_k12, g.plan1d, g.plan2,
                   static_cast<const cplx<T>*>(g.tw1), static_cast<const cplx<T>*>(g.tw2), out);
}

bool k2d_inverse_applies(const Geometry& g, int nocc) {
  // 72 x 72 planes: the accumulators of a 108 x 108 plane would not fit in registers
  return plane_static(g) == 72 && nocc % 2 == 0;
}

template <typename T>
bool launch_k2d_inverse(const Geometry& g, const cplx<T>* dst, int nrows, int r0, int nocc,
                        const T* phi, T alpha, T* R, hipStream_t s) {
  if (!k2d_inverse_applies(g, nocc)) return false;
  WTD_REQUIRE(nrows >= 1 && r0 >= 0 && r0 + nrows <= nocc, WTD_ERR_SHAPE,
              "K2d row chunk out of range");
  dim3 grid((unsigned)((g.n0 * (nocc / 2) + 7) / 8 * 8));
  const size_t lds = (size_t)g.plane * sizeof(cplx<T>);
  WTD_PLANE_LAUNCH(k_k2d_inverse, T, grid, lds, s, dst, nrows, r0, nocc, g.n0, g.n1, g.n2, g.nd,
                   g.nds, g.dst_k12, g.plan1d, g.plan2, static_cast<const cplx<T>*>(g.tw1),
                   static_cast<const cplx<T>*>(g.tw2), phi, alpha, R);
  return true;
}

template <typename T>
void launch_fields_to_wsticks(const Geometry& g, const T* fields, int nb, int per_trial,
                              int nfield_per_trial, cplx<T>* wst, hipStream_t s) {
  (void)nfield_per_trial;
  const int npt = (per_trial + 1) / 2;
  const int npack = nb * npt;
  if (g.quad_sn > 0) {
    WTD_QUAD_LAUNCH(k_fields_to_wsticks_q, T, g.nwrow, g.n0 * npack, s, fields, npt, per_trial,
                    g.n0, g.nws, g.nwrow, g.wrows, wst, npack);
    return;
  }
  const int items = plane_static(g) > 0 ? kPairItems : 1;
  const int ngrp = (g.n0 * npack + items - 1) / items;
  dim3 grid((unsigned)((ngrp + 7) / 8 * 8));
  const size_t lds = (size_t)g.plane * sizeof(cplx<T>);
  WTD_PLANE_LAUNCH(k_fields_to_wsticks, T, grid, lds, s, fields, npt, per_trial, items, g.n0,
                   g.n1, g.n2, g.nw, g.nws, g.wst_k12, g.plan1w, g.plan2,
                   static_cast<const cplx<T>*>(g.tw1), static_cast<const cplx<T>*>(g.tw2), wst,
                   npack);
}

template <typename T>
void launch_wsticks_to_sphere(const Geometry& g, cplx<T>* wst, int npack, hipStream_t s) {
  dim3 grid((g.nw + kStickTile - 1) / kStickTile, npack);
  const size_t lds = (size_t)g.n0 * kStickTile * sizeof(cplx<T>);
  WTD_STICK_LAUNCH(k_wsticks_forward, T, grid, lds, s, wst, g.n0, g.nw, g.nws, g.plan0,
                   static_cast<const cplx<T>*>(g.tw0));
}

template <typename T>
void launch_extract_sphere(const Geometry& g, const cplx<T>* wst, int nb, int per_trial,
                           int nfield_per_trial, int npw, T scale, T* coef, hipStream_t s) {
  (void)nfield_per_trial;
  const int npt = (per_trial + 1) / 2;
  dim3 grid((npw + 255) / 256, nb * npt);
  hipLaunchKernelGGL(k_extract_sphere<T>, grid, dim3(256), 0, s, wst, npt, per_trial, g.n0, g.nws,
                     npw, g.sph_pos, scale, coef);
  WTD_HIP(hipGetLastError());
}

template <typename T>
void launch_contract(const Geometry& g, int nb, int nocc, const T* phi, const T* at,
                     const T* tau, const int* pair_index, const T* vh, const T* drho,
                     const T* fxc, T ck, T alpha, bool k1e, bool k1d, T* R, hipStream_t s) {
  const int ntile = (int)((g.nr + kCtPts - 1) / kCtPts);
  const int nvb = (nocc + kCtV - 1) / kCtV;
  const int ntile8 = (ntile + 7) / 8 * 8;
  const int64_t nblk = (int64_t)ntile8 * nvb;
  WTD_REQUIRE(nblk < (1ll << 31), WTD_ERR_SHAPE, "contraction grid too large");
  hipLaunchKernelGGL(k_contract<T>, dim3((unsigned)nblk), dim3(256), 0, s, nb, nocc, g.nr, ntile,
                     nvb, phi, at, tau, pair_index, vh, drho, fxc, ck, alpha, (int)k1e, (int)k1d,
                     R);
  WTD_HIP(hipGetLastError());
}

template <typename T>
void launch_dterm_combine(int nb, int nocc, int nc, const T* S, const T* Q, const double* eo,
                          const double* ec, bool with_d, T* out, hipStream_t s) {
  const int64_t tot = (int64_t)nb * nocc * nc;
  hipLaunchKernelGGL(k_dterm_combine<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     nb, nocc, nc, S, Q, eo, ec, (int)with_d, out);
  WTD_HIP(hipGetLastError());
}

template <typename Tin, typename Tout>
void launch_convert(const Tin* in, Tout* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     in, out, n);
  WTD_HIP(hipGetLastError());
}

template <typename T>
void launch_zero(T* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL((k_zero<T>), dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  WTD_HIP(hipGetLastError());
}

template void launch_zero<float>(float*, int64_t, hipStream_t);
template void launch_zero<double>(double*, int64_t, hipStream_t);

namespace {
// flag = 1 if any of x[0..n) is a NaN or an infinity (flag zeroed beforehand)
template <typename T>
__global__ void k_flag_nonfinite(const T* __restrict__ x, int64_t n, unsigned* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad = bad || !isfinite(x[i]);
  if (bad) atomicOr(flag, 1u);
}
}  // namespace

template <typename T>
void launch_flag_nonfinite(const T* x, int64_t n, unsigned* flag, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL((k_flag_nonfinite<T>), dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
  WTD_HIP(hipGetLastError());
}

template void launch_flag_nonfinite<float>(const float*, int64_t, unsigned*, hipStream_t);
template void launch_flag_nonfinite<double>(const double*, int64_t, unsigned*, hipStream_t);

void launch_transition_out(int nb, int nocc, int nc, const void* Q, bool q_is_float,
                           const double* X, const double* eo, const double* ec, bool with_d,
                           double* T, hipStream_t s) {
  const int64_t tot = (int64_t)nb * nocc * nc;
  hipLaunchKernelGGL(k_transition_out, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nb,
                     nocc, nc, Q, (int)q_is_float, X, eo, ec, (int)with_d, T);
  WTD_HIP(hipGetLastError());
}

#define WTD_INST(T)                                                                            \
  template void launch_sphere_to_wsticks<T>(const Geometry&, const T*, int, int, int, int,     \
                                            cplx<T>*, hipStream_t);                            \
  template void launch_wsticks_to_fields<T>(const Geometry&, const cplx<T>*, int, int, int, T, \
                                            T*, const T*, T*, hipStream_t, T*, int);           \
  template void launch_pairs_to_dsticks<T>(const Geometry&, const T*, const int4*, int, int,   \
                                           cplx<T>*, hipStream_t);                             \
  template void launch_dstick_poisson<T>(const Geometry&, cplx<T>*, int, hipStream_t);         \
  template void launch_dsticks_to_fields<T>(const Geometry&, const cplx<T>*, int, int, T*,     \
                                            hipStream_t, bool);                                \
  template bool launch_k2d_inverse<T>(const Geometry&, const cplx<T>*, int, int, int, const T*, \
                                      T, T*, hipStream_t);                                     \
  template void launch_fields_to_wsticks<T>(const Geometry&, const T*, int, int, int,          \
                                            cplx<T>*, hipStream_t);                            \
  template void launch_wsticks_to_sphere<T>(const Geometry&, cplx<T>*, int, hipStream_t);      \
  template void launch_extract_sphere<T>(const Geometry&, const cplx<T>*, int, int, int, int,  \
                                         T, T*, hipStream_t);                                  \
  template void launch_contract<T>(const Geometry&, int, int, const T*, const T*, const T*,    \
                                   const int*, const T*, const T*, const T*, T, T, bool, bool, \
                                   T*, hipStream_t);                                           \
  template void launch_dterm_combine<T>(int, int, int, const T*, const T*, const double*,      \
                                        const double*, bool, T*, hipStream_t);

WTD_INST(float)
WTD_INST(double)

template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);

}  // namespace wtd
