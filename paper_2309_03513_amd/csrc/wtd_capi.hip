// C ABI, context set-up and the host-side schedule of the Liouville apply.
//
// Apply schedule for a block of nb trial sets (the paper's Sec. 2.1 terms; all
// device work on the context stream):
//   1. S = Phi_c^T a                        (MFMA GEMM, weighted Gamma inner product)
//   2. a~ = Phi_c S                         (MFMA GEMM): projected input
//   3. a~(r) and drho_b = sum_v phi_v a~_bv (stick + plane pass, fused reduction)
//   4. v_H,b = v_c * drho_b                 (Poisson on density sticks)       [K1e]
//   5. tau_vv' = v_c * (phi_v phi_v'), v <= v' (packed pair Poisson)          [K1d]
//   6. R_bv = c_K phi_v (v_H,b + f_xc drho_b) - alpha sum_v' tau_vv' a~_bv'
//   7. r_bv = sphere coefficients of R_bv   (plane + stick pass, unpacking)
//   8. Q = Phi_c^T r ; T = (eps_c - eps_v) S + Q ; la = Phi_c T
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "wtd_internal.h"

namespace wtd {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

// ---------------------------------------------------------------- device memory
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Profiler {
  bool on = false;
  static constexpr int kStages = 11;
  const char* names[kStages] = {"project_in",     "trial_to_grid", "hartree",
                                "pair_plane_fwd", "pair_stick_poisson", "pair_plane_inv",
                                "contract",       "grid_to_sphere", "project_out",
                                "davidson_small", "k2d"};
  double ms[kStages] = {};
  int64_t calls[kStages] = {};
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;  // (stage, index of start event)
};

}  // namespace

}  // namespace wtd

struct wtd_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  wtd_precision prec = WTD_FP64;
  uint32_t mask = WTD_TERM_ALL;
  int npw = 0, nocc = 0, nc = 0, max_nb = 0;
  double alpha = 0, ck = 0, vg0 = 0;
  wtd::Geometry g{};
  std::vector<double> eps_occ_h, eps_cond_h;
  std::vector<wtd::DevBuf> bufs;
  size_t total_bytes = 0;
  // device arrays (precision-typed as void*)
  void* c_cond = nullptr;    // [nc][2 npw]
  void* c_condw = nullptr;   // weighted copy for the Gamma inner product
  void* c_occ = nullptr;     // [nocc][2 npw]
  double* eps_occ = nullptr;
  double* eps_cond = nullptr;
  double* diag = nullptr;    // [nocc*nc] eps_c - eps_v (Davidson preconditioner)
  void* fxc = nullptr;
  void* phi = nullptr;       // [nocc][nr]
  void* at = nullptr;        // [max_nb][nocc][nr]
  void* R = nullptr;         // [max_nb][nocc][nr]
  void* drho = nullptr;      // [max_nb][nr]
  void* vh = nullptr;        // [max_nb][nr]
  void* drho_part = nullptr; // [8][max_nb][nr] partial densities
  void* tau = nullptr;       // [npairs][nr]
  // Pair potentials depend on the occupied orbitals only: with tau_cache on they
  // are kept from one apply to the next until the orbitals change.
  bool tau_cache = false;
  bool tau_valid = false;
  // layout the kept pair potentials were written in (4-pair interleaved or
  // [pair][N_r]); a later apply that reads the other layout forms them again
  bool tau_il = false;
  // all pairs kept in the tile order of the round-robin contraction
  // (rr_tile_base) rather than row-major
  bool tile_pairs = false;
  // The all-pairs potentials depend on the orbitals only: an apply that forms
  // them does so on pair_stream (default priority), forked from the context
  // stream at the apply's start and joined before the contraction, so the
  // projection, trial transform and Hartree solve run beside them.
  // In FP64 the pair chunks themselves are pipelined over two streams and two
  // stick buffers: chunk k + 1's forward plane pass on pair_stream while chunk
  // k's stick Poisson and inverse plane pass run on pair_stream2 (FP64 72^3
  // apply 48.3 -> 46.8 ms; in FP32, where the forward and inverse plane
  // kernels share the LDS of a CU, 19.64 -> 19.89 ms, so FP32 keeps one pair
  // stream).
  hipStream_t pair_stream = nullptr, pair_stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_fwd[2] = {}, ev_free[2] = {};
  bool pairs_pending = false;  // pairs enqueued on the pair streams, not yet joined
  int last_fwd = 0;            // ev_fwd slot recorded last on pair_stream
  void* dsth = nullptr;        // density sticks of the Hartree solve ((max_nb + 1) / 2 packs)
  void* dst2 = nullptr;        // second stick buffer of the pipelined pair chunks
  void* wst = nullptr;       // [max packs][n0][nw] complex
  void* dst = nullptr;       // [pair chunk][n0][nd] complex
  void* ag = nullptr;        // [max_nb][nocc][2 npw]
  void* rg = nullptr;        // [max_nb][nocc][2 npw]
  void* S = nullptr;         // [max_nb*nocc][nc]
  void* Q = nullptr;
  void* Tm = nullptr;
  void* gemm_scratch = nullptr;  // split-K partial products
  size_t gemm_scratch_elems = 0;
  int npairs = 0, npack_pairs = 0, pair_chunk = 0;
  int max_pair_chunk = 0;    // packs the density-stick buffer holds
  int drho_groups = 8;       // workgroups per trial of the density reduction
  int4* quads = nullptr;     // pair packs
  int4* hquads = nullptr;    // Hartree packs
  // K2d packs: products a_bv' phi_v of trial b, pair q = v' nocc + v, two per pack;
  // field indices count phi (nocc fields) then the trial fields (max_nb * nocc)
  int4* k2quads = nullptr;   // [max_nb][k2_npk]
  int k2_npk = 0;
  size_t tau_fields = 0;     // fields the pair-potential buffer holds
  // backward-only buffers, allocated on the first backward call
  bool bwd_ready = false;
  void* gt = nullptr;        // [max_nb][nocc][nr] cotangent fields g~
  void* drhog = nullptr;     // [max_nb][nr]
  void* vhg = nullptr;       // [max_nb][nr]
  void* gamma = nullptr;     // [nocc][nr]
  void* gbuf = nullptr;      // [max_nb][nocc][2 npw]
  int4* pquads = nullptr;    // packs of stored pair fields (2p, 2p+1)
  int* pidx = nullptr;       // [nocc][nocc]
  // Row-blocked exchange (large Nocc): the pair triangle is split into blocks of
  // row_block occupied rows; tau then holds the pairs of one block pair only.
  uint32_t checks = 0;       // WTD_CHECK_* flags of wtd_set_checks
  unsigned* flag = nullptr;  // device word of the non-finite check
  int row_block = 0;         // 0: all pairs at once
  struct BlockPair {
    int A0, nA, B0, nB, diag;
    int q0, npairs, npack;   // packs quads[q0 .. q0 + npack)
  };
  std::vector<BlockPair> bpairs;
  wtd::Profiler prof;
  // this device's copy of the static Davidson scratch array (wtd_davidson_noalloc)
  void* scratch = nullptr;
};

namespace wtd {

namespace {

// groups over which the orbital loop of the trial transform is split
constexpr int kDrhoGroups = 8;

// Device memory of wtd_davidson_noalloc, for callers that cannot allocate: one
// statically sized array that every GPU the library runs on holds until the
// process ends.  Its name is only a host-side stand-in; host code passes the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = WTD_DAVIDSON_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of its copy of scratch

// Address of the scratch array on `device`, which must be the current device.
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    throw StatusError{WTD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e)};
  }
  g_scratch_ptr.emplace(device, ptr);
  return ptr;
}

// device memory one context may hold (wtd_set_workspace_limit; 0: no cap)
std::atomic<size_t> g_workspace_limit{0};

void* dalloc(wtd_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 16;
  const size_t cap = g_workspace_limit.load();
  if (cap != 0 && c->total_bytes + bytes > cap)
    throw StatusError{WTD_ERR_OOM, "context workspace would exceed the limit of " +
                                       std::to_string(cap) + " bytes (" +
                                       std::to_string(c->total_bytes + bytes) + " needed so far)"};
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError{WTD_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  c->bufs.push_back({p, bytes});
  c->total_bytes += bytes;
  return p;
}

void free_all(wtd_ctx* c) {
  if (c->pair_stream) (void)hipStreamSynchronize(c->pair_stream);
  for (auto& b : c->bufs) (void)hipFree(b.p);
  c->bufs.clear();
  if (c->pair_stream2) (void)hipStreamSynchronize(c->pair_stream2);
  for (hipEvent_t* e : {&c->ev_fork, &c->ev_join, &c->ev_fwd[0], &c->ev_fwd[1], &c->ev_free[0],
                        &c->ev_free[1]}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  if (c->pair_stream) (void)hipStreamDestroy(c->pair_stream);
  if (c->pair_stream2) (void)hipStreamDestroy(c->pair_stream2);
  c->pair_stream = c->pair_stream2 = nullptr;
  for (auto e : c->prof.pool) (void)hipEventDestroy(e);
  c->prof.pool.clear();
}

// Host-to-device copy that has completed when it returns (the source may be a
// temporary).
void h2d(wtd_ctx* c, void* dst, const void* src, size_t bytes) {
  WTD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  WTD_HIP(hipStreamSynchronize(c->stream));
}

template <typename T>
void upload(wtd_ctx* c, void* dst, const std::vector<T>& h) {
  h2d(c, dst, h.data(), h.size() * sizeof(T));
}

// Synchronous scan of a device array for NaN / infinity: WTD_ERR_NONFINITE names it.
template <typename T>
void require_finite(wtd_ctx* c, const T* x, int64_t n, const char* what) {
  WTD_HIP(hipMemsetAsync(c->flag, 0, sizeof(unsigned), c->stream));
  launch_flag_nonfinite<T>(x, n, c->flag, c->stream);
  unsigned h = 0;
  WTD_HIP(hipMemcpyAsync(&h, c->flag, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  WTD_HIP(hipStreamSynchronize(c->stream));
  WTD_REQUIRE(h == 0, WTD_ERR_NONFINITE, std::string("non-finite values in ") + what);
}

void require_finite_any(wtd_ctx* c, const void* x, int64_t n, const char* what) {
  if (c->prec == WTD_FP64)
    require_finite<double>(c, (const double*)x, n, what);
  else
    require_finite<float>(c, (const float*)x, n, what);
}

// ---------------------------------------------------------------- profiling
void prof_mark(wtd_ctx* c, int stage) {
  if (!c->prof.on) return;
  Profiler& P = c->prof;
  while (P.pool.size() < P.used + 2) {
    hipEvent_t e;
    WTD_HIP(hipEventCreate(&e));
    P.pool.push_back(e);
  }
  WTD_HIP(hipEventRecord(P.pool[P.used], c->stream));
  P.marks.push_back({stage, P.used});
  P.used += 2;
}

void prof_end(wtd_ctx* c) {
  if (!c->prof.on || c->prof.marks.empty()) return;
  Profiler& P = c->prof;
  WTD_HIP(hipEventRecord(P.pool[P.marks.back().second + 1], c->stream));
}

// Close the current stage and open the next one.
void prof_next(wtd_ctx* c, int stage) {
  if (!c->prof.on) return;
  Profiler& P = c->prof;
  if (!P.marks.empty()) {
    const size_t idx = P.marks.back().second + 1;
    WTD_HIP(hipEventRecord(P.pool[idx], c->stream));
  }
  prof_mark(c, stage);
}

// Sum the recorded stage intervals (synchronises on the last event).
void prof_collect(wtd_ctx* c) {
  Profiler& P = c->prof;
  if (P.marks.empty()) return;
  WTD_HIP(hipEventSynchronize(P.pool[P.marks.back().second + 1]));
  for (auto& m : P.marks) {
    float ms = 0.f;
    WTD_HIP(hipEventElapsedTime(&ms, P.pool[m.second], P.pool[m.second + 1]));
    P.ms[m.first] += ms;
    P.calls[m.first] += 1;
  }
  P.marks.clear();
  P.used = 0;
}

// Called at the end of an operation: events are kept until wtd_profile_read,
// unless the pool grows large.
void prof_finish(wtd_ctx* c) {
  if (!c->prof.on) return;
  if (c->prof.marks.size() > 4096) prof_collect(c);
}

// ---------------------------------------------------------------- geometry
FFTPlan make_plan(int n) {
  FFTPlan P{};
  P.n = n;
  P.cut = -1;
  int rem = n, np = 0, prod = 1;
  const int order[] = {8, 5, 4, 3, 2};
  while (rem > 1) {
    int r = 0;
    for (int cand : order)
      if (rem % cand == 0) {
        r = cand;
        break;
      }
    WTD_REQUIRE(r != 0, WTD_ERR_SHAPE,
                "grid size " + std::to_string(n) + " is not a product of 2, 3 and 5");
    WTD_REQUIRE(np < kMaxPasses, WTD_ERR_SHAPE, "too many FFT passes");
    P.rad[np] = r;
    P.p[np] = prod;
    prod *= r;
    rem /= r;
    ++np;
  }
  P.np = np;
  return P;
}

int fold(int m, int n) { return ((m % n) + n) % n; }
int unfold(int k, int n) { return (2 * k < n) ? k : k - n; }

template <typename T>
void* make_twiddles(wtd_ctx* c, int n) {
  std::vector<T> h(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)n;
    h[2 * j] = (T)std::cos(a);
    h[2 * j + 1] = (T)(-std::sin(a));
  }
  void* d = dalloc(c, h.size() * sizeof(T));
  upload(c, d, h);
  return d;
}

template <typename T>
void build_geometry(wtd_ctx* c, const wtd_system* sys) {
  Geometry& g = c->g;
  g.n0 = sys->n[0];
  g.n1 = sys->n[1];
  g.n2 = sys->n[2];
  g.plane = g.n1 * g.n2;
  g.nr = (int64_t)g.n0 * g.plane;
  g.omega = sys->cell[0] * sys->cell[1] * sys->cell[2];
  g.plan0 = make_plan(g.n0);
  g.plan1 = make_plan(g.n1);
  g.plan2 = make_plan(g.n2);
  g.tw0 = make_twiddles<T>(c, g.n0);
  g.tw1 = make_twiddles<T>(c, g.n1);
  g.tw2 = make_twiddles<T>(c, g.n2);
  const int n[3] = {g.n0, g.n1, g.n2};
  const double b[3] = {2 * M_PI / sys->cell[0], 2 * M_PI / sys->cell[1], 2 * M_PI / sys->cell[2]};

  // validate the half sphere
  const int npw = sys->npw;
  const int32_t* mill = sys->mill;
  WTD_REQUIRE(mill[0] == 0 && mill[1] == 0 && mill[2] == 0, WTD_ERR_SHAPE,
              "the first Miller index must be m = 0");
  std::set<std::tuple<int, int, int>> seen;
  double g2max = 0.0;
  for (int h = 0; h < npw; ++h) {
    const int m0 = mill[3 * h], m1 = mill[3 * h + 1], m2 = mill[3 * h + 2];
    for (int i = 0; i < 3; ++i)
      WTD_REQUIRE(2 * std::abs(mill[3 * h + i]) < n[i], WTD_ERR_SHAPE,
                  "grid too small for the plane-wave sphere (need n_i > 2 max|m_i|)");
    if (h > 0) {
      const int first = m0 != 0 ? m0 : (m1 != 0 ? m1 : m2);
      WTD_REQUIRE(first > 0, WTD_ERR_SHAPE, "Miller index outside the Gamma half space");
    }
    WTD_REQUIRE(seen.insert({m0, m1, m2}).second, WTD_ERR_SHAPE, "duplicate Miller index");
    const double g2 = (m0 * b[0]) * (m0 * b[0]) + (m1 * b[1]) * (m1 * b[1]) +
                      (m2 * b[2]) * (m2 * b[2]);
    g2max = std::max(g2max, g2);
  }

  // wave sticks: columns (k1, k2) holding +m or -m
  std::map<int, int> wkey;
  for (int h = 0; h < npw; ++h)
    for (int sg = -1; sg <= 1; sg += 2) {
      const int k1 = fold(sg * mill[3 * h + 1], n[1]), k2 = fold(sg * mill[3 * h + 2], n[2]);
      wkey[k1 * n[2] + k2] = 0;
    }
  std::vector<int> wk12;
  for (auto& kv : wkey) {
    kv.second = (int)wk12.size();
    wk12.push_back(kv.first);
  }
  g.nw = (int)wk12.size();
  // stick rows start on 128-byte boundaries, so the 16-stick tiles of the
  // stick kernels never share a cache line
  g.nws = (g.nw + 15) / 16 * 16;
  g.nwtile = (g.nw + kStickTile - 1) / kStickTile;
  std::vector<std::vector<int4>> tiles(g.nwtile);
  std::vector<int> pos(2 * (size_t)npw);
  for (int h = 0; h < npw; ++h) {
    for (int sg = 1; sg >= -1; sg -= 2) {
      if (h == 0 && sg < 0) {
        pos[2 * h + 1] = pos[2 * h];
        continue;
      }
      const int k0 = fold(sg * mill[3 * h], n[0]);
      const int k1 = fold(sg * mill[3 * h + 1], n[1]), k2 = fold(sg * mill[3 * h + 2], n[2]);
      const int s = wkey[k1 * n[2] + k2];
      tiles[s / kStickTile].push_back(int4{h, sg, s % kStickTile, k0});
      pos[2 * h + (sg > 0 ? 0 : 1)] = k0 * g.nws + s;
    }
  }
  std::vector<int> off(g.nwtile + 1, 0);
  std::vector<int4> ent;
  for (int t = 0; t < g.nwtile; ++t) {
    off[t] = (int)ent.size();
    ent.insert(ent.end(), tiles[t].begin(), tiles[t].end());
  }
  off[g.nwtile] = (int)ent.size();
  int* d_wk = (int*)dalloc(c, wk12.size() * sizeof(int));
  upload(c, d_wk, wk12);
  int* d_off = (int*)dalloc(c, off.size() * sizeof(int));
  upload(c, d_off, off);
  int4* d_ent = (int4*)dalloc(c, ent.size() * sizeof(int4));
  h2d(c, d_ent, ent.data(), ent.size() * sizeof(int4));
  int2* d_pos = (int2*)dalloc(c, pos.size() * sizeof(int));
  upload(c, d_pos, pos);
  g.wst_k12 = d_wk;
  g.wtile_off = d_off;
  g.wtile_ent = d_ent;
  g.sph_pos = d_pos;

  // density sticks: projections of |G| <= 2 max|G_sphere| (pair products), folded
  std::set<int> dkey;
  const int r1 = (int)std::floor(2.0 * std::sqrt(g2max) / b[1]) + 1;
  const int r2 = (int)std::floor(2.0 * std::sqrt(g2max) / b[2]) + 1;
  for (int m1 = -r1; m1 <= r1; ++m1)
    for (int m2 = -r2; m2 <= r2; ++m2) {
      const double gg = (m1 * b[1]) * (m1 * b[1]) + (m2 * b[2]) * (m2 * b[2]);
      if (gg <= 4.0 * g2max * (1.0 + 1e-12)) dkey.insert(fold(m1, n[1]) * n[2] + fold(m2, n[2]));
    }
  std::vector<int> dk12(dkey.begin(), dkey.end());
  g.nd = (int)dk12.size();
  g.nds = (g.nd + 15) / 16 * 16;
  int* d_dk = (int*)dalloc(c, dk12.size() * sizeof(int));
  upload(c, d_dk, dk12);
  g.dst_k12 = d_dk;
  // rows of the stick sets for the register-quad plane kernels
  auto stick_rows = [&](const std::vector<int>& k12, int& nrow, const int4*& dev, int& rmax) {
    std::vector<int4> rows;
    bool regular = true;
    rmax = -1;
    const int ns = (int)k12.size();
    for (int s0 = 0; s0 < ns;) {
      const int k1 = k12[s0] / n[2];
      int s1 = s0;
      while (s1 < ns && k12[s1] / n[2] == k1) ++s1;
      const int cnt = s1 - s0, R = (cnt - 1) / 2;
      bool ok = cnt % 2 == 1 && 2 * R + 1 <= n[2];
      for (int i = 0; ok && i < cnt; ++i)
        ok = k12[s0 + i] % n[2] == (i <= R ? i : n[2] - (cnt - i));
      regular = regular && ok;
      rmax = std::max(rmax, R);
      rows.push_back(int4{k1, s0, R, 0});
      s0 = s1;
    }
    nrow = regular ? (int)rows.size() : 0;
    if (!regular) rmax = -1;
    int4* d = (int4*)dalloc(c, std::max<size_t>(rows.size(), 1) * sizeof(int4));
    if (!rows.empty()) h2d(c, d, rows.data(), rows.size() * sizeof(int4));
    dev = d;
  };
  int dcut = -1, wcut = -1;
  stick_rows(dk12, g.ndrow, g.drows, dcut);
  stick_rows(wk12, g.nwrow, g.wrows, wcut);
  // column passes of the density- and wave-stick plane kernels: only the
  // columns k2 their stick rows reach (every column if the rows are irregular
  // or the plane is not square)
  g.plan1d = g.plan1;
  g.plan1w = g.plan1;
  if (g.n1 == g.n2) {
    g.plan1d.cut = (dcut >= 0 && 2 * dcut + 1 < g.n2) ? dcut : -1;
    g.plan1w.cut = (wcut >= 0 && 2 * wcut + 1 < g.n2) ? wcut : -1;
  }
  {
    const char* e = std::getenv("WTD_QUAD_PLANES");
    g.quad_sn = quad_plane_size(g, sizeof(T), e && std::atoi(e) != 0);
  }
  std::vector<T> kern((size_t)g.nd * g.n0);
  for (int s = 0; s < g.nd; ++s) {
    const int m1 = unfold(dk12[s] / n[2], n[1]), m2 = unfold(dk12[s] % n[2], n[2]);
    for (int k0 = 0; k0 < g.n0; ++k0) {
      const int m0 = unfold(k0, n[0]);
      const double gg = (m0 * b[0]) * (m0 * b[0]) + (m1 * b[1]) * (m1 * b[1]) +
                        (m2 * b[2]) * (m2 * b[2]);
      const double v = gg > 0.0 ? 4.0 * M_PI / gg : c->vg0;
      kern[(size_t)s * g.n0 + k0] = (T)(v / (double)g.nr);
    }
  }
  void* d_kern = dalloc(c, kern.size() * sizeof(T));
  upload(c, d_kern, kern);
  g.dkern = d_kern;
}

// ---------------------------------------------------------------- context set-up
template <typename T>
void create_impl(wtd_ctx* c, const wtd_system* sys) {
  build_geometry<T>(c, sys);
  const int npw = c->npw, nocc = c->nocc, nc = c->nc, mnb = c->max_nb;
  const int64_t nr = c->g.nr;
  const size_t K = 2 * (size_t)npw;
  hipStream_t s = c->stream;

  // every system array must be finite
  c->flag = (unsigned*)dalloc(c, sizeof(unsigned));
  for (int v = 0; v < nocc; ++v)
    WTD_REQUIRE(std::isfinite(sys->eps_occ[v]), WTD_ERR_NONFINITE, "non-finite eps_occ");
  for (int ci = 0; ci < nc; ++ci)
    WTD_REQUIRE(std::isfinite(sys->eps_cond[ci]), WTD_ERR_NONFINITE, "non-finite eps_cond");
  require_finite<double>(c, sys->c_occ, (int64_t)nocc * K, "c_occ");
  require_finite<double>(c, sys->c_cond, (int64_t)nc * K, "c_cond");
  if (sys->fxc) require_finite<double>(c, sys->fxc, nr, "fxc");

  // orbitals in the working precision; weighted conduction copy for <phi_c|.>
  c->c_occ = dalloc(c, (size_t)nocc * K * sizeof(T));
  c->c_cond = dalloc(c, (size_t)nc * K * sizeof(T));
  c->c_condw = dalloc(c, (size_t)nc * K * sizeof(T));
  {
    std::vector<double> hc((size_t)nc * K);
    WTD_HIP(hipMemcpyAsync(hc.data(), sys->c_cond, hc.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    WTD_HIP(hipStreamSynchronize(s));
    std::vector<T> a(hc.size()), w(hc.size());
    for (int ci = 0; ci < nc; ++ci)
      for (int h = 0; h < npw; ++h) {
        const size_t i = (size_t)ci * K + 2 * h;
        a[i] = (T)hc[i];
        a[i + 1] = (h == 0) ? T(0) : (T)hc[i + 1];
        const double wt = (h == 0) ? 1.0 : 2.0;
        w[i] = (T)(wt * hc[i]);
        w[i + 1] = (h == 0) ? T(0) : (T)(wt * hc[i + 1]);
      }
    upload(c, c->c_cond, a);
    upload(c, c->c_condw, w);
    WTD_HIP(hipStreamSynchronize(s));
  }
  c->eps_occ = (double*)dalloc(c, nocc * sizeof(double));
  c->eps_cond = (double*)dalloc(c, nc * sizeof(double));
  upload(c, c->eps_occ, c->eps_occ_h);
  upload(c, c->eps_cond, c->eps_cond_h);
  {
    std::vector<double> d((size_t)nocc * nc);
    for (int v = 0; v < nocc; ++v)
      for (int ci = 0; ci < nc; ++ci) d[(size_t)v * nc + ci] = c->eps_cond_h[ci] - c->eps_occ_h[v];
    c->diag = (double*)dalloc(c, d.size() * sizeof(double));
    upload(c, c->diag, d);
  }
  c->fxc = dalloc(c, nr * sizeof(T));
  if (sys->fxc) {
    if (sizeof(T) == sizeof(double))
      WTD_HIP(hipMemcpyAsync(c->fxc, sys->fxc, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    else
      launch_convert<double, float>(sys->fxc, (float*)c->fxc, nr, s);
  } else {
    WTD_HIP(hipMemsetAsync(c->fxc, 0, nr * sizeof(T), s));
  }

  // the trial transform that forms the density response keeps a grid plane in
  // LDS, and with runtime FFT plans also its real accumulator
  if ((c->mask & (WTD_TERM_K1E | WTD_TERM_K2E)) && c->ck != 0.0 && c->g.quad_sn == 0) {
    const bool reg_acc = plane_static_wave(c->g) > 0;
    WTD_REQUIRE((size_t)c->g.plane * (sizeof(cplx<T>) + (reg_acc ? 0 : sizeof(T))) +
                        108 * sizeof(cplx<T>) <= 160 * 1024,
                WTD_ERR_SHAPE,
                "the density response needs a grid plane (and, with runtime FFT plans, its "
                "accumulator) in 160 KB of LDS (FP64: planes up to 96 x 96 with compile-time "
                "plans, about 80 x 80 otherwise; FP32: up to 108 x 108)");
  }
  // pairs v <= v' (row-major), packed two per complex transform
  c->npairs = nocc * (nocc + 1) / 2;
  c->npack_pairs = (c->npairs + 1) / 2;
  // Above 128 occupied orbitals the pair triangle is processed in blocks of 64
  // rows; so is every FP32 system the all-pairs round-robin contraction does
  // not cover (Nocc != 128 or blocks not of whole 16-trial tiles), whose
  // register-operand block contraction is the faster one there
  // (WTD_ROW_BLOCK = 16, 32, 48 or 64 selects blocking for any Nocc).
  const bool rr = c->prec == WTD_FP32 && nocc == 128 && mnb % 16 == 0 && nr % 8 == 0;
  c->row_block = (nocc > 128 || (c->prec == WTD_FP32 && !rr)) ? 64 : 0;
  if (const char* e = std::getenv("WTD_ROW_BLOCK")) {
    const int rb = std::atoi(e);
    WTD_REQUIRE(rb >= 0 && rb <= 64 && rb % 16 == 0, WTD_ERR_ARG,
                "WTD_ROW_BLOCK must be 0, 16, 32, 48 or 64");
    if (rb > 0) c->row_block = rb;
  }
  // (planes too large for LDS run the register-quad kernels, which write
  // [pair][N_r] fields only)
  c->tile_pairs = c->row_block == 0 && c->g.quad_sn == 0 && contract_rr_applies<T>(c->g, mnb, nocc);
  {
    std::vector<int2> pr;
    std::vector<int> pidx;
    std::vector<int4> q;
    auto pack = [&](size_t first) {
      for (size_t p = first; p < pr.size(); p += 2) {
        const int2 a = pr[p];
        const int2 b = (p + 1 < pr.size()) ? pr[p + 1] : int2{-1, -1};
        q.push_back(int4{a.x, a.y, b.x, b.y});
      }
    };
    auto add_pair = [&](int v, int w) {
      pidx[(size_t)v * nocc + w] = pidx[(size_t)w * nocc + v] = (int)pr.size();
      pr.push_back(int2{v, w});
    };
    if (c->tile_pairs) {
      // 16 x 16 row tiles (I <= J) in the order the round-robin contraction
      // addresses them: diagonal tiles as upper triangles, row by row
      pidx.resize((size_t)nocc * nocc);
      for (int I = 0; I < nocc / 16; ++I)
        for (int J = I; J < nocc / 16; ++J) {
          WTD_REQUIRE((int)pr.size() == rr_tile_base(I, J), WTD_ERR_SHAPE,
                      "pair tile order");
          for (int a = 0; a < 16; ++a)
            for (int b = (I == J) ? a : 0; b < 16; ++b) add_pair(16 * I + a, 16 * J + b);
        }
      pack(0);
    } else if (c->row_block == 0) {
      pidx.resize((size_t)nocc * nocc);
      for (int v = 0; v < nocc; ++v)
        for (int w = v; w < nocc; ++w) add_pair(v, w);
      pack(0);
    } else {
      // block pairs (A, B), A <= B; the diagonal block stores its upper
      // triangle row-major, an off-diagonal block its full rectangle
      const int rb = c->row_block;
      for (int A0 = 0; A0 < nocc; A0 += rb)
        for (int B0 = A0; B0 < nocc; B0 += rb) {
          wtd_ctx::BlockPair bp;
          bp.A0 = A0;
          bp.nA = std::min(rb, nocc - A0);
          bp.B0 = B0;
          bp.nB = std::min(rb, nocc - B0);
          bp.diag = A0 == B0;
          const size_t first = pr.size();
          for (int i = 0; i < bp.nA; ++i)
            for (int j = bp.diag ? i : 0; j < bp.nB; ++j) pr.push_back(int2{A0 + i, B0 + j});
          bp.q0 = (int)q.size();
          bp.npairs = (int)(pr.size() - first);
          pack(first);
          bp.npack = (int)q.size() - bp.q0;
          c->bpairs.push_back(bp);
        }
      pidx.resize(1);
    }
    c->quads = (int4*)dalloc(c, q.size() * sizeof(int4));
    h2d(c, c->quads, q.data(), q.size() * sizeof(int4));
    c->pidx = (int*)dalloc(c, pidx.size() * sizeof(int));
    upload(c, c->pidx, pidx);
    std::vector<int4> hq((mnb + 1) / 2);
    for (int p = 0; p < (int)hq.size(); ++p)
      hq[p] = int4{2 * p, -1, (2 * p + 1 < mnb) ? 2 * p + 1 : -1, -1};
    c->hquads = (int4*)dalloc(c, hq.size() * sizeof(int4));
    h2d(c, c->hquads, hq.data(), hq.size() * sizeof(int4));
    WTD_HIP(hipStreamSynchronize(s));
  }

  // workspace
  const int npt = (nocc + 1) / 2;
  const size_t nwp = (size_t)std::max(mnb * npt, npt);
  // phi and the projected trial fields share one allocation, so that pair
  // kernels can form products of a trial field and an orbital (K2d)
  c->phi = dalloc(c, ((size_t)nocc + (size_t)mnb * nocc) * nr * sizeof(T));
  c->at = (T*)c->phi + (size_t)nocc * nr;
  c->R = dalloc(c, (size_t)mnb * nocc * nr * sizeof(T));
  c->drho = dalloc(c, (size_t)mnb * nr * sizeof(T));
  c->vh = dalloc(c, (size_t)mnb * nr * sizeof(T));
  c->drho_part = dalloc(c, (size_t)kDrhoGroups * mnb * nr * sizeof(T));
  // (rounded up to whole groups of 8 for the interleaved layout)
  const size_t tau_fields =
      ((c->row_block ? std::min<size_t>((size_t)c->row_block * c->row_block, c->npairs)
                     : (size_t)c->npairs) + 7) / 8 * 8;
  if (c->alpha != 0.0 && (c->mask & (WTD_TERM_K1D | WTD_TERM_K2D))) {
    c->tau = dalloc(c, tau_fields * nr * sizeof(T));
    c->tau_fields = tau_fields;
  }
  if (c->alpha != 0.0 && (c->mask & WTD_TERM_K2D)) {
    const int64_t nq = (int64_t)nocc * nocc;
    c->k2_npk = (int)((nq + 1) / 2);
    std::vector<int4> kq((size_t)mnb * c->k2_npk);
    for (int b = 0; b < mnb; ++b) {
      const int A = nocc + b * nocc;
      for (int64_t k = 0; k < c->k2_npk; ++k) {
        const int64_t q0 = 2 * k, q1 = 2 * k + 1;
        int4 e{A + (int)(q0 / nocc), (int)(q0 % nocc), -1, -1};
        if (q1 < nq) e.z = A + (int)(q1 / nocc), e.w = (int)(q1 % nocc);
        kq[(size_t)b * c->k2_npk + k] = e;
      }
    }
    c->k2quads = (int4*)dalloc(c, kq.size() * sizeof(int4));
    h2d(c, c->k2quads, kq.data(), kq.size() * sizeof(int4));
  }
  c->wst = dalloc(c, nwp * c->g.n0 * c->g.nws * sizeof(cplx<T>));
  // packed pairs per Poisson batch; the density-stick intermediate of one batch
  // is batch * n0 * n_d complex values (WTD_PAIR_CHUNK overrides the default)
  int chunk = 512;
  if (const char* e = std::getenv("WTD_PAIR_CHUNK")) chunk = std::max(1, std::atoi(e));
  c->pair_chunk = std::max(1, std::min(c->npack_pairs, chunk));
  // chunks start on whole groups of 8 fields (4 packs) for the interleaved layout
  if (c->pair_chunk >= 4) c->pair_chunk = c->pair_chunk / 4 * 4;
  if (c->row_block) {
    c->pair_chunk = std::min(c->pair_chunk, (int)((tau_fields + 1) / 2));
    if (c->pair_chunk >= 4) c->pair_chunk = c->pair_chunk / 4 * 4;
  }
  c->max_pair_chunk = c->pair_chunk;
  const int dchunk = std::max(c->pair_chunk, (mnb + 1) / 2);
  c->dst = dalloc(c, (size_t)dchunk * c->g.n0 * c->g.nds * sizeof(cplx<T>));
  c->dsth = dalloc(c, (size_t)((mnb + 1) / 2) * c->g.n0 * c->g.nds * sizeof(cplx<T>));
  if (!c->row_block && sizeof(T) == 8)
    c->dst2 = dalloc(c, (size_t)c->pair_chunk * c->g.n0 * c->g.nds * sizeof(cplx<T>));
  WTD_HIP(hipStreamCreateWithFlags(&c->pair_stream, hipStreamNonBlocking));
  WTD_HIP(hipStreamCreateWithFlags(&c->pair_stream2, hipStreamNonBlocking));
  for (hipEvent_t* e : {&c->ev_fork, &c->ev_join, &c->ev_fwd[0], &c->ev_fwd[1], &c->ev_free[0],
                        &c->ev_free[1]})
    WTD_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  c->ag = dalloc(c, (size_t)mnb * nocc * K * sizeof(T));
  c->rg = dalloc(c, (size_t)mnb * nocc * K * sizeof(T));
  c->S = dalloc(c, (size_t)mnb * nocc * nc * sizeof(T));
  c->Q = dalloc(c, (size_t)mnb * nocc * nc * sizeof(T));
  c->Tm = dalloc(c, (size_t)mnb * nocc * nc * sizeof(T));
  c->gemm_scratch_elems = (size_t)16 * mnb * nocc * nc;
  c->gemm_scratch = dalloc(c, c->gemm_scratch_elems * sizeof(T));
}

template <typename T>
void transform_occ(wtd_ctx* c, const double* c_occ) {
  const int nocc = c->nocc, npw = c->npw;
  const size_t K = 2 * (size_t)npw;
  hipStream_t s = c->stream;
  if (sizeof(T) == sizeof(double))
    WTD_HIP(hipMemcpyAsync(c->c_occ, c_occ, (size_t)nocc * K * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  else
    launch_convert<double, float>(c_occ, (float*)c->c_occ, (int64_t)nocc * K, s);
  launch_sphere_to_wsticks<T>(c->g, (const T*)c->c_occ, nocc, npw, 1, nocc, (cplx<T>*)c->wst, s);
  launch_wsticks_to_fields<T>(c->g, (const cplx<T>*)c->wst, 1, nocc, nocc,
                              (T)(1.0 / std::sqrt(c->g.omega)), (T*)c->phi, nullptr, nullptr, s);
}

// ---------------------------------------------------------------- the apply (steps 3-7)
// Input: S [nb*nocc][nc] and a~ in G space (ag); output Q [nb*nocc][nc].
// mask: the terms to apply (WTD_TERM_*; K2e and K2d only for the full operator).
// At the Gamma point the trial fields are real, so K2e's density
// sum_v' conj(a_v') phi_v' equals K1e's and the two add up to one response term.
// The all-pairs potentials are kept from an earlier apply (pair cache on).
bool pairs_kept(const wtd_ctx* c) {
  return c->tau_cache && c->tau_valid && c->tau_il == c->tile_pairs;
}

// Step 5 for all pairs at once, on stream s: pair potentials in chunks of
// packed pairs, stored interleaved by groups of kTauIl pairs in the tile order
// of the round-robin contraction where it reads them (a chunk starts on a
// whole group, so its groups start at field 2 p0 in either layout).
template <typename T>
void form_pairs(wtd_ctx* c, hipStream_t s) {
  const Geometry& g = c->g;
  const bool il = c->tile_pairs;
  WTD_REQUIRE(!il || (2 * c->pair_chunk) % kTauIl == 0 || c->pair_chunk >= c->npack_pairs,
              WTD_ERR_SHAPE, "pair chunk must be a multiple of 2 packs (whole groups of 4 pairs)");
  for (int p0 = 0; p0 < c->npack_pairs; p0 += c->pair_chunk) {
    const int np = std::min(c->pair_chunk, c->npack_pairs - p0);
    const int nf = std::min(2 * np, c->npairs - 2 * p0);
    prof_next(c, 3);
    launch_pairs_to_dsticks<T>(g, (const T*)c->phi, c->quads + p0, np, c->nocc,
                               (cplx<T>*)c->dst, s);
    prof_next(c, 4);
    launch_dstick_poisson<T>(g, (cplx<T>*)c->dst, np, s);
    prof_next(c, 5);
    launch_dsticks_to_fields<T>(g, (const cplx<T>*)c->dst, np, nf,
                                (T*)c->tau + (int64_t)2 * p0 * g.nr, s, il);
  }
  c->tau_valid = c->tau_cache;
  c->tau_il = il;
}

// The same pipelined over the two pair streams and the two stick buffers
// (events order each buffer's reuse after the inverse pass that read it).
template <typename T>
void form_pairs_pipelined(wtd_ctx* c) {
  const Geometry& g = c->g;
  const bool il = c->tile_pairs;
  WTD_REQUIRE(!il || (2 * c->pair_chunk) % kTauIl == 0 || c->pair_chunk >= c->npack_pairs,
              WTD_ERR_SHAPE, "pair chunk must be a multiple of 2 packs (whole groups of 4 pairs)");
  hipStream_t sf = c->pair_stream, sp = c->pair_stream2;
  cplx<T>* buf[2] = {(cplx<T>*)c->dst, (cplx<T>*)c->dst2};
  int k = 0;
  for (int p0 = 0; p0 < c->npack_pairs; p0 += c->pair_chunk, ++k) {
    const int b = k & 1;
    const int np = std::min(c->pair_chunk, c->npack_pairs - p0);
    const int nf = std::min(2 * np, c->npairs - 2 * p0);
    if (k >= 2) WTD_HIP(hipStreamWaitEvent(sf, c->ev_free[b], 0));
    launch_pairs_to_dsticks<T>(g, (const T*)c->phi, c->quads + p0, np, c->nocc, buf[b], sf);
    WTD_HIP(hipEventRecord(c->ev_fwd[b], sf));
    WTD_HIP(hipStreamWaitEvent(sp, c->ev_fwd[b], 0));
    launch_dstick_poisson<T>(g, buf[b], np, sp);
    launch_dsticks_to_fields<T>(g, buf[b], np, nf, (T*)c->tau + (int64_t)2 * p0 * g.nr, sp, il);
    WTD_HIP(hipEventRecord(c->ev_free[b], sp));
    c->last_fwd = b;
  }
  c->tau_valid = c->tau_cache;
  c->tau_il = il;
}

// The context stream waits for the pair work forked by fork_pairs (both pair
// streams end in it).
void join_pairs(wtd_ctx* c) {
  if (!c->pairs_pending) return;
  if (c->last_fwd >= 0) WTD_HIP(hipStreamWaitEvent(c->stream, c->ev_fwd[c->last_fwd], 0));
  WTD_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
  c->pairs_pending = false;
}

// Joins the forked pair work when an apply stops with an error between its
// fork and its join (the normal path joins before the contraction), so that no
// later work on the context stream overlaps it.
struct PairJoinOnError {
  wtd_ctx* c;
  ~PairJoinOnError() {
    try {
      join_pairs(c);
    } catch (...) {
      // (the error that unwound the apply is the one reported)
    }
  }
};

// At the start of an apply: enqueue the all-pairs potentials on the pair
// streams after the work already on the context stream (they read only the
// orbital fields), to be joined before the contraction.  Not with stage
// profiling (its events time one stream) nor with WTD_PAIR_OVERLAP=0.
template <typename T>
void fork_pairs(wtd_ctx* c, uint32_t mask) {
  static const bool off = [] {
    const char* e = std::getenv("WTD_PAIR_OVERLAP");
    return e && std::atoi(e) == 0;
  }();
  const bool k1d = (mask & WTD_TERM_K1D) && c->alpha != 0.0;
  if (off || !k1d || c->row_block || c->prof.on || pairs_kept(c)) return;
  // under stream capture the chunks stay on one pair stream: the two-stream
  // pipeline (events re-recorded and waited on across both forked streams)
  // crashed the capture's end, which the one-stream form does not
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  WTD_HIP(hipStreamIsCapturing(c->stream, &cap));
  WTD_HIP(hipEventRecord(c->ev_fork, c->stream));
  WTD_HIP(hipStreamWaitEvent(c->pair_stream, c->ev_fork, 0));
  if (c->dst2 && cap == hipStreamCaptureStatusNone) {
    WTD_HIP(hipStreamWaitEvent(c->pair_stream2, c->ev_fork, 0));
    form_pairs_pipelined<T>(c);
    WTD_HIP(hipEventRecord(c->ev_join, c->pair_stream2));
  } else {
    form_pairs<T>(c, c->pair_stream);
    WTD_HIP(hipEventRecord(c->ev_join, c->pair_stream));
    c->last_fwd = -1;
  }
  c->pairs_pending = true;
}

template <typename T>
void apply_core(wtd_ctx* c, int nb, uint32_t mask) {
  const Geometry& g = c->g;
  hipStream_t s = c->stream;
  const int nocc = c->nocc, npw = c->npw, nc = c->nc;
  const int K = 2 * npw;
  const int nresp = ((mask & WTD_TERM_K1E) ? 1 : 0) + ((mask & WTD_TERM_K2E) ? 1 : 0);
  const double ck = c->ck * nresp;
  const bool k1e = nresp > 0 && c->ck != 0.0;
  const bool k1d = (mask & WTD_TERM_K1D) && c->alpha != 0.0;
  const bool k2d = (mask & WTD_TERM_K2D) && c->alpha != 0.0;
  const int F = nb * nocc;
  if (!k1e && !k1d && !k2d) {
    launch_zero<T>((T*)c->Q, (int64_t)F * nc, s);
    return;
  }
  const int npt = (nocc + 1) / 2;
  // 3. trial transform (+ density response)
  prof_next(c, 1);
  launch_sphere_to_wsticks<T>(g, (const T*)c->ag, F, npw, nb, nocc, (cplx<T>*)c->wst, s);
  launch_wsticks_to_fields<T>(g, (const cplx<T>*)c->wst, nb, nocc, nocc,
                              (T)(1.0 / std::sqrt(g.omega)), (T*)c->at, (const T*)c->phi,
                              k1e ? (T*)c->drho : nullptr, s, (T*)c->drho_part, c->drho_groups);
  // 4. Hartree potential of drho_b
  if (k1e) {
    prof_next(c, 2);
    const int nh = (nb + 1) / 2;
    launch_pairs_to_dsticks<T>(g, (const T*)c->drho, c->hquads, nh, nb, (cplx<T>*)c->dsth, s);
    launch_dstick_poisson<T>(g, (cplx<T>*)c->dsth, nh, s);
    launch_dsticks_to_fields<T>(g, (const cplx<T>*)c->dsth, nh, nb, (T*)c->vh, s);
  }
  if (c->row_block) {
    // 5'-6'. R = response term, then the exchange sum block pair by block pair
    prof_next(c, 6);
    launch_response_rows<T>(g, nb, nocc, (const T*)c->phi, (const T*)c->vh, (const T*)c->drho,
                            (const T*)c->fxc, (T)ck, k1e, (T*)c->R, s);
    if (k1d) {
      // FP32: pair potentials in the interleaved layout and the register-operand
      // block contraction
      const bool bil = contract_block_rr_applies<T>(nb);
      int max_npack = 0;
      for (const auto& bp : c->bpairs) max_npack = std::max(max_npack, bp.npack);
      WTD_REQUIRE(!bil || c->pair_chunk % 2 == 0 || c->pair_chunk >= max_npack, WTD_ERR_SHAPE,
                  "pair chunk must start on whole groups of 4 pairs");
      // one block pair holds every pair: its potentials can be kept between applies
      const bool single = c->bpairs.size() == 1;
      const bool reuse = single && c->tau_cache && c->tau_valid;
      for (const auto& bp : c->bpairs) {
        for (int p0 = 0; p0 < (reuse ? 0 : bp.npack); p0 += c->pair_chunk) {
          const int np = std::min(c->pair_chunk, bp.npack - p0);
          const int nf = std::min(2 * np, bp.npairs - 2 * p0);
          prof_next(c, 3);
          launch_pairs_to_dsticks<T>(g, (const T*)c->phi, c->quads + bp.q0 + p0, np, c->nocc,
                                     (cplx<T>*)c->dst, s);
          prof_next(c, 4);
          launch_dstick_poisson<T>(g, (cplx<T>*)c->dst, np, s);
          prof_next(c, 5);
          launch_dsticks_to_fields<T>(g, (const cplx<T>*)c->dst, np, nf,
                                      (T*)c->tau + (int64_t)2 * p0 * g.nr, s, bil);
        }
        if (single) c->tau_valid = c->tau_cache;
        prof_next(c, 6);
        if (bil)
          launch_contract_block_rr<T>(g, nb, nocc, (const T*)c->at, (const T*)c->tau, bp.A0,
                                      bp.nA, bp.B0, bp.nB, bp.diag != 0, (T)c->alpha, (T*)c->R,
                                      s);
        else
          launch_contract_block<T>(g, nb, nocc, (const T*)c->at, (const T*)c->tau, bp.A0, bp.nA,
                                   bp.B0, bp.nB, bp.diag != 0, (T)c->alpha, (T*)c->R, s);
      }
    }
  }
  // 5. pair potentials: joined from pair_stream, or formed here
  if (c->pairs_pending) {
    join_pairs(c);
  } else if (k1d && !c->row_block && !pairs_kept(c)) {
    form_pairs<T>(c, s);
  }
  const bool il = c->tile_pairs;
  // 6. R
  prof_next(c, 6);
  if (c->row_block) {
  } else if (!k1e && !k1d) {
    launch_zero<T>((T*)c->R, (int64_t)nb * nocc * g.nr, s);
  } else if (!launch_contract_mfma<T>(g, nb, nocc, (const T*)c->phi, (const T*)c->at, (const T*)c->tau,
                               (const T*)c->vh, (const T*)c->drho, (const T*)c->fxc, (T)ck,
                               (T)c->alpha, k1e, k1d, (T*)c->R, s, il))
    launch_contract<T>(g, nb, nocc, (const T*)c->phi, (const T*)c->at, (const T*)c->tau, c->pidx,
                       (const T*)c->vh, (const T*)c->drho, (const T*)c->fxc, (T)ck,
                       (T)c->alpha, k1e, k1d, (T*)c->R, s);
  // 6b. K2d: R_bv -= alpha sum_v' phi_v' v_c * (a_bv' phi_v), trial by trial, in
  // chunks of rows v' whose nocc pair fields fit in the pair-potential buffer
  if (k2d) {
    prof_next(c, 10);
    c->tau_valid = false;
    const int nfield_all = nocc * (1 + c->max_nb);
    int rows = (int)std::min<size_t>((size_t)nocc, c->tau_fields / (size_t)nocc);
    if (rows < nocc && (nocc & 1)) rows &= ~1;  // chunks start on whole packs
    WTD_REQUIRE(rows >= 1, WTD_ERR_SHAPE, "pair buffer too small for one row of K2d pairs");
    // 72 x 72 planes and even Nocc: the Poisson-solved products of as many
    // rows as the pair buffer holds as density sticks are formed first, then
    // transformed back and contracted by one fused kernel (no W fields)
    const size_t cap_packs = c->tau_fields * (size_t)g.nr / 2 / ((size_t)g.n0 * g.nds);
    const int hp = nocc / 2;
    const int rows_f = k2d_inverse_applies(g, nocc) ? (int)std::min<size_t>(nocc, cap_packs / hp) : 0;
    const bool fused = rows_f >= 1;
    for (int b = 0; fused && b < nb; ++b) {
      const int4* kq = c->k2quads + (size_t)b * c->k2_npk;
      for (int r0 = 0; r0 < nocc; r0 += rows_f) {
        const int nrw = std::min(rows_f, nocc - r0);
        const int npk = nrw * hp;
        const int k0 = r0 * hp;
        cplx<T>* sticks = (cplx<T>*)c->tau;
        for (int p0 = 0; p0 < npk; p0 += c->pair_chunk) {
          const int np = std::min(c->pair_chunk, npk - p0);
          cplx<T>* d = sticks + (int64_t)p0 * g.n0 * g.nds;
          launch_pairs_to_dsticks<T>(g, (const T*)c->phi, kq + k0 + p0, np, nfield_all, d, s);
          launch_dstick_poisson<T>(g, d, np, s);
        }
        WTD_REQUIRE(launch_k2d_inverse<T>(g, sticks, nrw, r0, nocc, (const T*)c->phi,
                                          (T)c->alpha, (T*)c->R + (int64_t)b * nocc * g.nr, s),
                    WTD_ERR_SHAPE, "fused K2d pass not applicable");
      }
    }
    for (int b = 0; !fused && b < nb; ++b) {
      const int4* kq = c->k2quads + (size_t)b * c->k2_npk;
      for (int r0 = 0; r0 < nocc; r0 += rows) {
        const int nrw = std::min(rows, nocc - r0);
        const int nf = nrw * nocc;
        const int k0 = (int)((int64_t)r0 * nocc / 2);
        const int npk = (nf + 1) / 2;
        for (int p0 = 0; p0 < npk; p0 += c->pair_chunk) {
          const int np = std::min(c->pair_chunk, npk - p0);
          const int nfs = std::min(2 * np, nf - 2 * p0);
          launch_pairs_to_dsticks<T>(g, (const T*)c->phi, kq + k0 + p0, np, nfield_all,
                                     (cplx<T>*)c->dst, s);
          launch_dstick_poisson<T>(g, (cplx<T>*)c->dst, np, s);
          launch_dsticks_to_fields<T>(g, (const cplx<T>*)c->dst, np, nfs,
                                      (T*)c->tau + (int64_t)2 * p0 * g.nr, s);
        }
        launch_k2d_rows<T>(g, nocc, nrw, r0, (const T*)c->phi, (const T*)c->tau, (T)c->alpha,
                           (T*)c->R + (int64_t)b * nocc * g.nr, s);
      }
    }
  }
  // 7. back to the sphere
  prof_next(c, 7);
  launch_fields_to_wsticks<T>(g, (const T*)c->R, nb, nocc, nocc, (cplx<T>*)c->wst, s);
  launch_wsticks_to_sphere<T>(g, (cplx<T>*)c->wst, nb * npt, s);
  launch_extract_sphere<T>(g, (const cplx<T>*)c->wst, nb, nocc, nocc, npw,
                           (T)(std::sqrt(g.omega) / (double)g.nr), (T*)c->rg, s);
  // 8a. Q = Phi_c^T r
  prof_next(c, 8);
  launch_gemm<T, true>(F, nc, K, (const T*)c->rg, K, (const T*)c->c_condw, K, (T*)c->Q, nc, s,
                       (T*)c->gemm_scratch, c->gemm_scratch_elems);
}

template <typename T>
void apply_impl(wtd_ctx* c, int nb, const T* a, T* la, uint32_t mask) {
  hipStream_t s = c->stream;
  const int nocc = c->nocc, npw = c->npw, nc = c->nc;
  const int K = 2 * npw, F = nb * nocc;
  prof_mark(c, 0);
  fork_pairs<T>(c, mask);
  PairJoinOnError join_on_error{c};
  launch_gemm<T, true>(F, nc, K, a, K, (const T*)c->c_condw, K, (T*)c->S, nc, s,
                       (T*)c->gemm_scratch, c->gemm_scratch_elems);
  launch_gemm<T, false>(F, K, nc, (const T*)c->S, nc, (const T*)c->c_cond, K, (T*)c->ag, K, s);
  apply_core<T>(c, nb, mask);
  prof_next(c, 8);
  launch_dterm_combine<T>(nb, nocc, nc, (const T*)c->S, (const T*)c->Q, c->eps_occ, c->eps_cond,
                          (mask & WTD_TERM_D) != 0, (T*)c->Tm, s);
  launch_gemm<T, false>(F, K, nc, (const T*)c->Tm, nc, (const T*)c->c_cond, K, la, K, s);
  prof_end(c);
  prof_finish(c);
}

template <typename T>
void apply_transition_impl(wtd_ctx* c, int nb, const double* X, double* Tout, uint32_t mask) {
  hipStream_t s = c->stream;
  const int nocc = c->nocc, npw = c->npw, nc = c->nc;
  const int K = 2 * npw, F = nb * nocc;
  prof_mark(c, 0);
  fork_pairs<T>(c, mask);
  PairJoinOnError join_on_error{c};
  if (sizeof(T) == sizeof(double))
    WTD_HIP(hipMemcpyAsync(c->S, X, (size_t)F * nc * sizeof(double), hipMemcpyDeviceToDevice, s));
  else
    launch_convert<double, float>(X, (float*)c->S, (int64_t)F * nc, s);
  launch_gemm<T, false>(F, K, nc, (const T*)c->S, nc, (const T*)c->c_cond, K, (T*)c->ag, K, s);
  apply_core<T>(c, nb, mask);
  prof_next(c, 8);
  launch_transition_out(nb, nocc, nc, c->Q, sizeof(T) == sizeof(float), X, c->eps_occ,
                        c->eps_cond, (mask & WTD_TERM_D) != 0, Tout, s);
  prof_end(c);
  prof_finish(c);
}

// the TDA operator: the context's D, K1e and K1d terms
uint32_t tda_mask(const wtd_ctx* c) { return c->mask & WTD_TERM_ALL; }

void apply_transition_any(wtd_ctx* c, int nb, const double* X, double* T, uint32_t mask) {
  if (c->prec == WTD_FP64)
    apply_transition_impl<double>(c, nb, X, T, mask);
  else
    apply_transition_impl<float>(c, nb, X, T, mask);
}

// ---------------------------------------------------------------- backward
template <typename T>
void bwd_prepare(wtd_ctx* c) {
  if (c->bwd_ready) return;
  const int64_t nr = c->g.nr;
  const int mnb = c->max_nb, nocc = c->nocc;
  c->gt = dalloc(c, (size_t)mnb * nocc * nr * sizeof(T));
  c->drhog = dalloc(c, (size_t)mnb * nr * sizeof(T));
  c->vhg = dalloc(c, (size_t)mnb * nr * sizeof(T));
  c->gamma = dalloc(c, (size_t)nocc * nr * sizeof(T));
  c->gbuf = dalloc(c, (size_t)mnb * nocc * 2 * c->npw * sizeof(T));
  std::vector<int4> q(c->npack_pairs);
  for (int p = 0; p < c->npack_pairs; ++p)
    q[p] = int4{2 * p, -1, (2 * p + 1 < c->npairs) ? 2 * p + 1 : -1, -1};
  c->pquads = (int4*)dalloc(c, q.size() * sizeof(int4));
  h2d(c, c->pquads, q.data(), q.size() * sizeof(int4));
  c->bwd_ready = true;
}

// v_c * of nf fields held at src (packed two per complex transform) into out
template <typename T>
void hartree_fields(wtd_ctx* c, const T* src, int nf, T* out) {
  const int nh = (nf + 1) / 2;
  launch_pairs_to_dsticks<T>(c->g, src, c->hquads, nh, nf, (cplx<T>*)c->dst, c->stream);
  launch_dstick_poisson<T>(c->g, (cplx<T>*)c->dst, nh, c->stream);
  launch_dsticks_to_fields<T>(c->g, (const cplx<T>*)c->dst, nh, nf, out, c->stream);
}

template <typename T>
void bwd_impl(wtd_ctx* c, int nb, const T* a, const T* g, T* g_a, T* g_occ) {
  const Geometry& G = c->g;
  hipStream_t s = c->stream;
  const int nocc = c->nocc, npw = c->npw, nc = c->nc;
  const int K = 2 * npw, F = nb * nocc;
  bwd_prepare<T>(c);
  if (g_a) {
    // dE/da = W L (W^-1 g)
    WTD_HIP(hipMemcpyAsync(c->gbuf, g, (size_t)F * K * sizeof(T), hipMemcpyDeviceToDevice, s));
    launch_weights<T>((T*)c->gbuf, F, npw, 0, s);
    apply_impl<T>(c, nb, (const T*)c->gbuf, g_a, tda_mask(c));
    launch_weights<T>(g_a, F, npw, 1, s);
  }
  if (!g_occ) return;
  const bool k1e = (c->mask & WTD_TERM_K1E) && c->ck != 0.0;
  const bool k1d = (c->mask & WTD_TERM_K1D) && c->alpha != 0.0;
  if (!k1e && !k1d) {
    launch_zero<T>(g_occ, (int64_t)nocc * K, s);
    return;
  }
  const T iso = (T)(1.0 / std::sqrt(G.omega));
  // projected trial fields a~(r) and drho
  launch_gemm<T, true>(F, nc, K, a, K, (const T*)c->c_condw, K, (T*)c->S, nc, s,
                       (T*)c->gemm_scratch, c->gemm_scratch_elems);
  launch_gemm<T, false>(F, K, nc, (const T*)c->S, nc, (const T*)c->c_cond, K, (T*)c->ag, K, s);
  launch_sphere_to_wsticks<T>(G, (const T*)c->ag, F, npw, nb, nocc, (cplx<T>*)c->wst, s);
  launch_wsticks_to_fields<T>(G, (const cplx<T>*)c->wst, nb, nocc, nocc, iso, (T*)c->at,
                              (const T*)c->phi, k1e ? (T*)c->drho : nullptr, s);
  // cotangent fields g~(r) = sum_c (phi_c . g) phi_c (Euclidean dot) and drho^g
  launch_gemm<T, true>(F, nc, K, g, K, (const T*)c->c_cond, K, (T*)c->Q, nc, s,
                       (T*)c->gemm_scratch, c->gemm_scratch_elems);
  launch_gemm<T, false>(F, K, nc, (const T*)c->Q, nc, (const T*)c->c_cond, K, (T*)c->rg, K, s);
  launch_sphere_to_wsticks<T>(G, (const T*)c->rg, F, npw, nb, nocc, (cplx<T>*)c->wst, s);
  launch_wsticks_to_fields<T>(G, (const cplx<T>*)c->wst, nb, nocc, nocc, iso, (T*)c->gt,
                              (const T*)c->phi, k1e ? (T*)c->drhog : nullptr, s);
  // exchange part: P_wv' = M_wv' + M_v'w -> v_c * P -> gamma = -alpha sum_v' phi_v' (v_c * P)
  // (the pair-density fields overwrite the pair potentials)
  if (k1d) c->tau_valid = false;
  if (k1d && c->row_block) {
    // gamma = -alpha sum_v' phi_v' v_c * P_wv', block pair by block pair
    launch_response_rows<T>(G, 1, nocc, (const T*)c->phi, nullptr, nullptr, nullptr, (T)0, false,
                            (T*)c->gamma, s);
    for (const auto& bp : c->bpairs) {
      launch_pair_density<T>(G, nb, nocc, (const T*)c->gt, (const T*)c->at, bp.A0, bp.nA, bp.B0,
                             bp.nB, bp.diag != 0, (T*)c->tau, s);
      const int npk = (bp.npairs + 1) / 2;
      for (int p0 = 0; p0 < npk; p0 += c->pair_chunk) {
        const int np = std::min(c->pair_chunk, npk - p0);
        const int nf = std::min(2 * np, bp.npairs - 2 * p0);
        launch_pairs_to_dsticks<T>(G, (const T*)c->tau + (int64_t)2 * p0 * G.nr, c->pquads, np,
                                   nf, (cplx<T>*)c->dst, s);
        launch_dstick_poisson<T>(G, (cplx<T>*)c->dst, np, s);
        launch_dsticks_to_fields<T>(G, (const cplx<T>*)c->dst, np, nf,
                                    (T*)c->tau + (int64_t)2 * p0 * G.nr, s);
      }
      launch_contract_block<T>(G, 1, nocc, (const T*)c->phi, (const T*)c->tau, bp.A0, bp.nA,
                               bp.B0, bp.nB, bp.diag != 0, (T)c->alpha, (T*)c->gamma, s);
    }
  } else if (k1d) {
    launch_pair_density<T>(G, nb, nocc, (const T*)c->gt, (const T*)c->at, 0, nocc, 0, nocc, true,
                           (T*)c->tau, s);
    for (int p0 = 0; p0 < c->npack_pairs; p0 += c->pair_chunk) {
      const int np = std::min(c->pair_chunk, c->npack_pairs - p0);
      const int nf = std::min(2 * np, c->npairs - 2 * p0);
      // pack p of this chunk holds stored pair fields 2 (p0 + p) and 2 (p0 + p) + 1
      launch_pairs_to_dsticks<T>(G, (const T*)c->tau + (int64_t)2 * p0 * G.nr, c->pquads, np, nf,
                                 (cplx<T>*)c->dst, s);
      launch_dstick_poisson<T>(G, (cplx<T>*)c->dst, np, s);
      launch_dsticks_to_fields<T>(G, (const cplx<T>*)c->dst, np, nf,
                                  (T*)c->tau + (int64_t)2 * p0 * G.nr, s);
    }
    if (!launch_contract_mfma<T>(G, 1, nocc, (const T*)c->phi, (const T*)c->phi,
                                 (const T*)c->tau, nullptr, nullptr, (const T*)c->fxc, (T)0,
                                 (T)c->alpha, false, true, (T*)c->gamma, s, false))
      launch_contract<T>(G, 1, nocc, (const T*)c->phi, (const T*)c->phi, (const T*)c->tau,
                         c->pidx, nullptr, nullptr, (const T*)c->fxc, (T)0, (T)c->alpha, false,
                         true, (T*)c->gamma, s);
  } else {
    launch_zero<T>((T*)c->gamma, (int64_t)nocc * G.nr, s);
  }
  // response part
  if (k1e) {
    hartree_fields<T>(c, (const T*)c->drho, nb, (T*)c->vh);
    hartree_fields<T>(c, (const T*)c->drhog, nb, (T*)c->vhg);
    launch_gamma_k1e<T>(G, nb, nocc, (T)c->ck, (const T*)c->gt, (const T*)c->at,
                        (const T*)c->vh, (const T*)c->drho, (const T*)c->vhg,
                        (const T*)c->drhog, (const T*)c->fxc, (T*)c->gamma, s);
  }
  // dE/dc_w(m) = (2 - delta_m0) coefficients of gamma_w
  const int npt = (nocc + 1) / 2;
  launch_fields_to_wsticks<T>(G, (const T*)c->gamma, 1, nocc, nocc, (cplx<T>*)c->wst, s);
  launch_wsticks_to_sphere<T>(G, (cplx<T>*)c->wst, npt, s);
  launch_extract_sphere<T>(G, (const cplx<T>*)c->wst, 1, nocc, nocc, npw,
                           (T)(std::sqrt(G.omega) / (double)G.nr), g_occ, s);
  launch_weights<T>(g_occ, nocc, npw, 1, s);
}

// ---------------------------------------------------------------- autotuner
// Times whole applies of an nb-trial block (zero input: the transforms and the
// contraction do the same work for any values) for each candidate setting and
// keeps the fastest by median of reps timed applies.
template <typename T>
void autotune_impl(wtd_ctx* c, int nb, int reps, int32_t* chunk_out, int32_t* groups_out) {
  hipStream_t s = c->stream;
  const size_t n = (size_t)nb * c->nocc * 2 * c->npw;
  struct Tmp {
    void* a = nullptr;
    void* la = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Tmp() {
      if (a) (void)hipFree(a);
      if (la) (void)hipFree(la);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } t;
  if (hipMalloc(&t.a, n * sizeof(T)) != hipSuccess || hipMalloc(&t.la, n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError{WTD_ERR_OOM, "autotuner trial block allocation failed"};
  }
  WTD_HIP(hipEventCreate(&t.e0));
  WTD_HIP(hipEventCreate(&t.e1));
  launch_zero<T>((T*)t.a, (int64_t)n, s);
  const bool prof_on = c->prof.on, cache_on = c->tau_cache;
  c->prof.on = false;
  c->tau_cache = false;
  auto time_apply = [&]() {
    apply_impl<T>(c, nb, (const T*)t.a, (T*)t.la, tda_mask(c));  // warm-up
    std::vector<float> ms(reps);
    for (int r = 0; r < reps; ++r) {
      WTD_HIP(hipEventRecord(t.e0, s));
      apply_impl<T>(c, nb, (const T*)t.a, (T*)t.la, tda_mask(c));
      WTD_HIP(hipEventRecord(t.e1, s));
      WTD_HIP(hipEventSynchronize(t.e1));
      WTD_HIP(hipEventElapsedTime(&ms[r], t.e0, t.e1));
    }
    std::sort(ms.begin(), ms.end());
    return ms[reps / 2];
  };
  try {
    // density split of the trial transform
    float best = 0.f;
    int best_g = c->drho_groups;
    for (int gs : {8, 4, 2, 1}) {
      c->drho_groups = gs;
      const float m = time_apply();
      if (gs == 8 || m < best) best = m, best_g = gs;
    }
    c->drho_groups = best_g;
    // packed pairs per Poisson batch: halvings of the allocated batch, whole
    // groups of 4 packs
    int best_c = c->pair_chunk;
    if (c->alpha != 0.0 && (c->mask & WTD_TERM_K1D)) {
      best = 0.f;
      bool first = true;
      for (int ch = c->max_pair_chunk; ch >= 16; ch /= 2) {
        const int cand = ch == c->max_pair_chunk ? ch : ch / 4 * 4;
        c->pair_chunk = cand;
        const float m = time_apply();
        if (first || m < best) best = m, best_c = cand;
        first = false;
      }
    }
    c->pair_chunk = best_c;
  } catch (...) {
    c->prof.on = prof_on;
    c->tau_cache = cache_on;
    c->tau_valid = false;
    throw;
  }
  c->prof.on = prof_on;
  c->tau_cache = cache_on;
  c->tau_valid = false;
  if (chunk_out) *chunk_out = c->pair_chunk;
  if (groups_out) *groups_out = c->drho_groups;
}

// ---------------------------------------------------------------- Davidson (FP64)
// Buffers of one Davidson or CG run: hipMalloc'ed and freed at the end, or (with
// an arena) carved from the static scratch array in 256-byte aligned pieces.
constexpr size_t dav_piece(size_t n) { return (std::max<size_t>(n, 2) * sizeof(double) + 255) / 256 * 256; }

struct DavWork {
  wtd_ctx* c;
  std::vector<void*> mem;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  ~DavWork() {
    for (void* p : mem) (void)hipFree(p);
  }
  double* alloc(size_t n) {
    if (arena) {
      const size_t b = dav_piece(n);
      if (used + b > cap)
        throw StatusError{WTD_ERR_SHAPE, "Davidson scratch exhausted (" +
                                             std::to_string(used + b) + " of " +
                                             std::to_string(cap) + " bytes)"};
      double* p = (double*)(arena + used);
      used += b;
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 2) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      throw StatusError{WTD_ERR_OOM, "Davidson workspace allocation failed"};
    }
    mem.push_back(p);
    return (double*)p;
  }
};

// Device bytes of the buffers davidson_impl takes (dav_piece each).
size_t davidson_need(const wtd_ctx* c, int nb, int max_sub, bool guess, bool want_x) {
  const size_t n = (size_t)c->nocc * c->nc, K = 2 * (size_t)c->npw, ms = max_sub;
  size_t t = 2 * dav_piece(ms * n)                 // V, W
             + dav_piece(ms * ms) + dav_piece(ms)   // H, evals
             + dav_piece(2 * ms * ms)               // evecs (+ rotation scratch)
             + dav_piece(ms * ms)                   // evecs transposed
             + 4 * dav_piece((size_t)nb * n)        // Ritz vectors, products, residuals, GEMM rows
             + dav_piece(nb)                        // residual norms
             + dav_piece((size_t)nb * ms)           // projection coefficients of a block
             + dav_piece(ms)                        // coefficients of one candidate
             + dav_piece(16 * ms * ms)              // split-K partial products
             + 2 * dav_piece(ms);                   // active list, slot flags (ints)
  if (guess) t += dav_piece((size_t)nb * n) + dav_piece((size_t)c->nc * K);
  if (want_x && c->prec != WTD_FP64) t += dav_piece((size_t)c->nc * K);
  return t;
}

// Block Davidson (Sec. 4).  Every iteration is one device-side step with no
// host synchronisation inside it: corrections of the roots that have not
// converged (the active list is formed on the device from the residual norms),
// their orthonormalisation against the basis (block Gram-Schmidt twice, as
// matrix-core GEMMs) and among themselves, the block apply, the subspace matrix
// V^T W (GEMM), its eigendecomposition, the Ritz vectors and products (GEMMs)
// and the residuals.  The host reads the Ritz values, residual norms and the
// kept/dropped flags of the new corrections once per iteration.  A correction
// whose norm falls below 1e-10 after orthogonalisation keeps its basis slot as
// a zero vector whose subspace diagonal is set to 1e30 (it never enters the
// lowest roots), so every step has a shape the host knows before it runs; on a
// non-null stream the step of each (basis size, block size) is captured once
// as a HIP graph and replayed.
// noalloc: every buffer comes from the static scratch array (no hipMalloc,
// hipFree or graph instantiation); the run is otherwise the same.
wtd_status davidson_impl(wtd_ctx* c, int nroots, int nb, double tol, int max_iter, int max_sub,
                         const double* guess, double* omega, double* x, double* resid,
                         int32_t* n_iter, bool noalloc = false) {
  hipStream_t s = c->stream;
  const int nocc = c->nocc, nc = c->nc, npw = c->npw;
  const int64_t n = (int64_t)nocc * nc;
  WTD_REQUIRE(n < (1ll << 31), WTD_ERR_SHAPE, "transition space too large");
  const int ni = (int)n;
  nb = (int)std::min<int64_t>(nb, n);
  if (max_sub <= 0) max_sub = 4 * nb;
  max_sub = std::max(max_sub, 2 * nb);
  max_sub = (int)std::min<int64_t>(max_sub, n);
  WTD_REQUIRE(max_sub <= 256, WTD_ERR_SHAPE, "max_sub must not exceed 256");
  DavWork w{c, {}};
  if (noalloc) {
    const size_t need = davidson_need(c, nb, max_sub, guess != nullptr, x != nullptr);
    WTD_REQUIRE(need <= kScratchBytes, WTD_ERR_SHAPE,
                "wtd_davidson_noalloc needs " + std::to_string(need) +
                    " bytes of scratch for this system and block (nocc*ncond = " +
                    std::to_string(n) + ", nb = " + std::to_string(nb) + ", max_sub = " +
                    std::to_string(max_sub) + "); the static array holds " +
                    std::to_string(kScratchBytes));
    WTD_REQUIRE(c->scratch != nullptr, WTD_ERR_HIP, "scratch array address not set");
    w.arena = (char*)c->scratch;
    w.cap = kScratchBytes;
  }
  // every apply of the run sees the same orbitals: form the pair potentials once
  struct KeepPairs {
    wtd_ctx* c;
    bool saved;
    ~KeepPairs() {
      c->tau_cache = saved;
      if (!saved) c->tau_valid = false;
    }
  } keep{c, c->tau_cache};
  if (!c->row_block || c->bpairs.size() == 1) c->tau_cache = true;
  const size_t ms = max_sub;
  double* V = w.alloc(ms * n);
  double* W = w.alloc(ms * n);
  double* H = w.alloc(ms * ms);
  double* evals = w.alloc(ms);
  double* evecs = w.alloc(2 * ms * ms);
  double* evecsT = w.alloc(ms * ms);
  double* Xr = w.alloc((size_t)nb * n);
  double* WY = w.alloc((size_t)nb * n);
  double* Rr = w.alloc((size_t)nb * n);
  double* tmp = w.alloc((size_t)nb * n);
  double* rn2 = w.alloc(nb);
  double* coefT = w.alloc((size_t)nb * ms);
  double* coef = w.alloc(ms);
  const size_t gscr_elems = 16 * ms * ms;
  double* gscr = w.alloc(gscr_elems);
  int* active = (int*)w.alloc(ms);
  int* ok = (int*)w.alloc(ms);

  // guess block in basis slots 0 .. nb-1
  if (guess) {
    // project the G-space guess onto transition coordinates: X = Phi_c^T g
    double* Sx = w.alloc((size_t)nb * n);
    double* Cw = w.alloc((size_t)nc * 2 * npw);
    if (c->prec == WTD_FP64) {
      launch_gemm<double, true>(nb * nocc, nc, 2 * npw, guess, 2 * npw, (const double*)c->c_condw,
                                2 * npw, Sx, nc, s);
    } else {
      launch_convert<float, double>((const float*)c->c_condw, Cw, (int64_t)nc * 2 * npw, s);
      launch_gemm<double, true>(nb * nocc, nc, 2 * npw, guess, 2 * npw, Cw, 2 * npw, Sx, nc, s);
    }
    WTD_HIP(hipMemcpyAsync(V, Sx, (size_t)nb * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    std::vector<int> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
      const int va = a / nc, ca = a % nc, vb = b / nc, cb = b % nc;
      const double da = c->eps_cond_h[ca] - c->eps_occ_h[va];
      const double db = c->eps_cond_h[cb] - c->eps_occ_h[vb];
      if (da != db) return da < db;
      if (ca != cb) return ca < cb;
      return va > vb;
    });
    std::vector<double> g((size_t)nb * n, 0.0);
    for (int j = 0; j < nb; ++j) g[(size_t)j * n + idx[j]] = 1.0;
    h2d(c, V, g.data(), g.size() * sizeof(double));
  }

  // rows T = V[m .. m + na): orthogonalised against V[0 .. m) twice (GEMMs),
  // then one by one against the rows before them (twice), then normalised or
  // dropped
  auto ortho_block = [&](int m, int na) {
    double* T = V + (int64_t)m * n;
    if (m > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        launch_gemm<double, true>(na, m, ni, T, ni, V, ni, coefT, m, s, gscr, gscr_elems);
        launch_gemm<double, false>(na, ni, m, coefT, m, V, ni, tmp, ni, s);
        launch_sub_rows(T, tmp, (int64_t)na * n, s);
      }
    }
    for (int j = 0; j < na; ++j) {
      double* t = T + (int64_t)j * n;
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        launch_gram(T, j, t, 1, n, coef, 1, s);
        launch_axpy_cols(t, T, coef, j, 1, n, s);
      }
      launch_normalise_or_drop(t, n, ok, m + j, s);
    }
  };
  // subspace of the first mt basis rows: H, eigenpairs, Ritz vectors, residuals
  auto finish = [&](int mt) {
    launch_gemm<double, true>(mt, mt, ni, V, ni, W, ni, H, max_sub, s, gscr, gscr_elems);
    launch_fix_dropped(H, max_sub, ok, mt, s);
    launch_jacobi_eig(H, mt, max_sub, evals, evecs, s);
    const int k = std::min(nb, mt);
    launch_transpose(evecs, mt, mt, evecsT, s);
    launch_gemm<double, false>(k, ni, mt, evecsT, mt, V, ni, Xr, ni, s);
    launch_gemm<double, false>(k, ni, mt, evecsT, mt, W, ni, WY, ni, s);
    launch_residual(WY, Xr, evals, k, n, Rr, rn2, s);
  };
  // one iteration after the first: corrections of the na active roots into
  // V[m .. m + na), their orthonormalisation, the apply and the new subspace
  const double tol2 = tol * tol;
  auto step = [&](int m, int na, int kprev) {
    launch_active_list(rn2, kprev, tol2, active, s);
    launch_precondition(Rr, evals, c->diag, na, n, active, V + (int64_t)m * n, s);
    ortho_block(m, na);
    apply_transition_any(c, na, V + (int64_t)m * n, W + (int64_t)m * n, tda_mask(c));
    finish(m + na);
  };

  struct Graphs {
    std::map<int, hipGraphExec_t> ex;
    ~Graphs() {
      for (auto& e : ex) (void)hipGraphExecDestroy(e.second);
    }
  } graphs;
  // (WTD_DAVIDSON_GRAPHS=0 runs every step eagerly; so does a run with
  // profiling on or on the null stream, which cannot be captured)
  bool use_graphs = !c->prof.on && s != nullptr && !noalloc;
  if (const char* e = std::getenv("WTD_DAVIDSON_GRAPHS")) use_graphs = use_graphs && std::atoi(e) != 0;
  auto run_step = [&](int m, int na, int kprev) {
    if (!use_graphs) {
      step(m, na, kprev);
      return;
    }
    const int key = (m * 512 + na) * 512 + kprev;
    auto it = graphs.ex.find(key);
    if (it == graphs.ex.end()) {
      hipGraph_t gr = nullptr;
      hipGraphExec_t ge = nullptr;
      WTD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        step(m, na, kprev);
      } catch (...) {
        (void)hipStreamEndCapture(s, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      WTD_HIP(hipStreamEndCapture(s, &gr));
      const hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      WTD_HIP(ie);
      it = graphs.ex.emplace(key, ge).first;
    }
    WTD_HIP(hipGraphLaunch(it->second, s));
  };

  std::vector<double> h_th(max_sub), h_rn2(nb), h_rn(nb);
  std::vector<int> h_ok(max_sub);
  {
    // an active list that is never read past its filled entries; zero it once
    std::vector<int> zeros(max_sub, 0);
    h2d(c, active, zeros.data(), zeros.size() * sizeof(int));
  }
  // read the Ritz values and residual norms of k roots and the flags of basis
  // rows [f0, f1)
  auto read_back = [&](int k, int f0, int f1) {
    WTD_HIP(hipMemcpyAsync(h_th.data(), evals, k * sizeof(double), hipMemcpyDeviceToHost, s));
    WTD_HIP(hipMemcpyAsync(h_rn2.data(), rn2, k * sizeof(double), hipMemcpyDeviceToHost, s));
    if (f1 > f0)
      WTD_HIP(hipMemcpyAsync(h_ok.data() + f0, ok + f0, (f1 - f0) * sizeof(int),
                             hipMemcpyDeviceToHost, s));
    WTD_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) h_rn[j] = std::sqrt(std::max(h_rn2[j], 0.0));
    int kept = 0;
    for (int j = f0; j < f1; ++j) kept += h_ok[j] != 0;
    return kept;
  };

  // first iteration: the guess block (eager: its apply forms the pair potentials)
  ortho_block(0, nb);
  apply_transition_any(c, nb, V, W, tda_mask(c));
  finish(nb);
  int m = nb;
  int kcur = std::min(nb, m);
  const int kept0 = read_back(kcur, 0, nb);
  WTD_REQUIRE(kept0 > 0, WTD_ERR_ARG, "Davidson guess block is rank deficient");
  int it = 0;
  bool converged = false;
  for (it = 1; it <= max_iter; ++it) {
    if (!std::isfinite(h_th[0])) throw StatusError{WTD_ERR_NONFINITE, "non-finite Ritz value"};
    // the same test on the same squared norms as the device's active list
    converged = true;
    for (int j = 0; j < std::min(nroots, kcur); ++j)
      if (!(h_rn2[j] <= tol2)) converged = false;
    if (converged || it == max_iter) break;
    int na = 0;
    for (int j = 0; j < kcur; ++j)
      if (h_rn2[j] > tol2) ++na;
    if (na == 0) throw StatusError{WTD_ERR_NONFINITE, "non-finite residual norm"};
    if (m + na > max_sub) {
      // restart from the current Ritz vectors
      WTD_HIP(hipMemcpyAsync(V, Xr, (size_t)kcur * n * sizeof(double), hipMemcpyDeviceToDevice, s));
      WTD_HIP(hipMemcpyAsync(W, WY, (size_t)kcur * n * sizeof(double), hipMemcpyDeviceToDevice, s));
      std::vector<int> ones(kcur, 1);
      h2d(c, ok, ones.data(), ones.size() * sizeof(int));
      m = kcur;
    }
    run_step(m, na, kcur);
    const int kept = read_back(std::min(nb, m + na), m, m + na);
    m += na;
    kcur = std::min(nb, m);
    if (kept == 0) break;  // every correction lies in the basis: it is exhausted
  }
  const int nr_out = std::min(nroots, kcur);
  for (int j = 0; j < nroots; ++j) {
    omega[j] = j < nr_out ? h_th[j] : NAN;
    if (resid) resid[j] = j < nr_out ? h_rn[j] : NAN;
  }
  if (n_iter) *n_iter = std::min(it, max_iter);
  if (x) {
    // x_k = Phi_c X_k in G space (FP64)
    const int K = 2 * npw;
    if (c->prec == WTD_FP64) {
      launch_gemm<double, false>(nr_out * nocc, K, nc, Xr, nc, (const double*)c->c_cond, K, x, K,
                                 s);
    } else {
      double* Cd = w.alloc((size_t)nc * K);
      launch_convert<float, double>((const float*)c->c_cond, Cd, (int64_t)nc * K, s);
      launch_gemm<double, false>(nr_out * nocc, K, nc, Xr, nc, Cd, K, x, K, s);
    }
  }
  WTD_HIP(hipStreamSynchronize(s));
  return converged ? WTD_OK : WTD_NOT_CONVERGED;
}

// ---------------------------------------------------------------- Z-vector CG (FP64)
// CG on the full operator in transition coordinates, nrhs systems side by side
// with their applies batched; each system drops K2d from its first iteration
// whose residual norm is below lambda_thr (inexact Krylov, Sec. 3.3).
wtd_status zvector_impl(wtd_ctx* c, int nrhs, const double* U, double tol, int max_iter,
                        double lambda_thr, double* Z, double* resid, int32_t* n_iter,
                        int32_t* n_exact) {
  hipStream_t s = c->stream;
  const int nocc = c->nocc, nc = c->nc, npw = c->npw, K = 2 * npw;
  const int64_t n = (int64_t)nocc * nc;
  DavWork w{c, {}};
  struct KeepPairs {
    wtd_ctx* c;
    bool saved;
    ~KeepPairs() {
      c->tau_cache = saved;
      if (!saved) c->tau_valid = false;
    }
  } keep{c, c->tau_cache};
  if (!c->row_block || c->bpairs.size() == 1) c->tau_cache = true;
  double* zt = w.alloc((size_t)nrhs * n);
  double* r = w.alloc((size_t)nrhs * n);
  double* p = w.alloc((size_t)nrhs * n);
  double* ap = w.alloc((size_t)nrhs * n);
  double* dots = w.alloc(nrhs);
  double* coef = w.alloc(nrhs);
  // right-hand sides in transition coordinates: b = Phi_c^T W U
  const double* cw = (const double*)c->c_condw;
  const double* cc = (const double*)c->c_cond;
  if (c->prec != WTD_FP64) {
    double* Cw = w.alloc((size_t)nc * K);
    double* Cd = w.alloc((size_t)nc * K);
    launch_convert<float, double>((const float*)c->c_condw, Cw, (int64_t)nc * K, s);
    launch_convert<float, double>((const float*)c->c_cond, Cd, (int64_t)nc * K, s);
    cw = Cw;
    cc = Cd;
  }
  launch_gemm<double, true>(nrhs * nocc, nc, K, U, K, cw, K, r, nc, s);
  launch_zero<double>(zt, (int64_t)nrhs * n, s);
  WTD_HIP(hipMemcpyAsync(p, r, (size_t)nrhs * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<double> rr(nrhs), pap(nrhs), rn(nrhs), hc(nrhs);
  launch_col_norms(r, nrhs, n, dots, s);
  WTD_HIP(hipMemcpyAsync(rr.data(), dots, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  WTD_HIP(hipStreamSynchronize(s));
  std::vector<char> active(nrhs);
  auto update_active = [&]() {
    bool any = false;
    for (int k = 0; k < nrhs; ++k) {
      if (!std::isfinite(rr[k])) throw StatusError{WTD_ERR_NONFINITE, "non-finite CG residual"};
      active[k] = std::sqrt(rr[k]) > tol;
      any = any || active[k];
    }
    return any;
  };
  // Each system switches to the operator without K2d on its own, at its first
  // iteration whose residual norm is below lambda_thr; per iteration the
  // systems still on the exact operator and those past their switch are
  // applied as two blocks (gathered into staging rows when not contiguous),
  // and converged systems get a zero product (their step is zero).
  std::vector<char> exact(nrhs, 1);
  double* ps = w.alloc((size_t)nrhs * n);
  double* aps = w.alloc((size_t)nrhs * n);
  auto apply_set = [&](const std::vector<int>& set, uint32_t mask) {
    if (set.empty()) return;
    const int m = (int)set.size();
    bool contiguous = true;
    for (int j = 1; j < m; ++j) contiguous = contiguous && set[j] == set[0] + j;
    if (contiguous) {
      apply_transition_any(c, m, p + (int64_t)set[0] * n, ap + (int64_t)set[0] * n, mask);
      return;
    }
    for (int j = 0; j < m; ++j)
      WTD_HIP(hipMemcpyAsync(ps + (int64_t)j * n, p + (int64_t)set[j] * n, n * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    apply_transition_any(c, m, ps, aps, mask);
    for (int j = 0; j < m; ++j)
      WTD_HIP(hipMemcpyAsync(ap + (int64_t)set[j] * n, aps + (int64_t)j * n, n * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  };
  int it = 0, nex = 0;
  while (update_active() && it < max_iter) {
    std::vector<int> on_exact, on_approx;
    for (int k = 0; k < nrhs; ++k) {
      if (!active[k]) {
        launch_zero<double>(ap + (int64_t)k * n, n, s);
        continue;
      }
      if (exact[k] && lambda_thr > 0.0 && std::sqrt(rr[k]) < lambda_thr) exact[k] = 0;
      (exact[k] ? on_exact : on_approx).push_back(k);
    }
    apply_set(on_exact, c->mask);
    apply_set(on_approx, c->mask & ~WTD_TERM_K2D);
    nex += on_exact.empty() ? 0 : 1;
    launch_col_dots(p, ap, nrhs, n, dots, s);
    WTD_HIP(hipMemcpyAsync(pap.data(), dots, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    WTD_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nrhs; ++k) {
      hc[k] = 0.0;
      if (!active[k]) continue;
      WTD_REQUIRE(pap[k] > 0.0 && std::isfinite(pap[k]), WTD_ERR_NONFINITE,
                  "CG breakdown: the operator is not positive definite on the search direction");
      hc[k] = rr[k] / pap[k];
    }
    h2d(c, coef, hc.data(), nrhs * sizeof(double));
    launch_cg_update(zt, r, p, ap, coef, nrhs, n, s);
    launch_col_norms(r, nrhs, n, dots, s);
    WTD_HIP(hipMemcpyAsync(rn.data(), dots, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    WTD_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nrhs; ++k) {
      hc[k] = active[k] ? rn[k] / rr[k] : 0.0;
      if (active[k]) rr[k] = rn[k];
    }
    h2d(c, coef, hc.data(), nrhs * sizeof(double));
    // frozen systems: beta = 0 turns p into r, which their zero step ignores
    launch_cg_direction(p, r, coef, nrhs, n, s);
    ++it;
  }
  bool converged = !update_active();
  for (int k = 0; k < nrhs; ++k)
    if (resid) resid[k] = std::sqrt(rr[k]);
  if (n_iter) *n_iter = it;
  if (n_exact) *n_exact = nex;
  // Z = Phi_c z in G space
  launch_gemm<double, false>(nrhs * nocc, K, nc, zt, nc, cc, K, Z, K, s);
  WTD_HIP(hipStreamSynchronize(s));
  return converged ? WTD_OK : WTD_NOT_CONVERGED;
}

template <typename F>
wtd_status guarded(F&& f) {
  try {
    return f();
  } catch (const StatusError& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return WTD_ERR_OOM;
  } catch (...) {
    set_error("unexpected internal error");
    return WTD_ERR_HIP;
  }
}

}  // namespace
}  // namespace wtd

using namespace wtd;

extern "C" {

const char* wtd_last_error(void) { return g_last_error.c_str(); }

wtd_status wtd_create(const wtd_system* sys, int32_t max_nb, void* hip_stream, wtd_ctx** out) {
  if (out) *out = nullptr;
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(sys && out, WTD_ERR_ARG, "null system or output pointer");
    WTD_REQUIRE(sys->mill && sys->c_occ && sys->c_cond && sys->eps_occ && sys->eps_cond,
                WTD_ERR_ARG, "null array in wtd_system");
    WTD_REQUIRE(max_nb >= 1, WTD_ERR_ARG, "max_nb must be >= 1");
    WTD_REQUIRE(sys->npw >= 1 && sys->nocc >= 1 && sys->ncond >= 1, WTD_ERR_SHAPE,
                "npw, nocc and ncond must be positive");
    WTD_REQUIRE(sys->n[0] >= 2 && sys->n[1] >= 2 && sys->n[2] >= 2, WTD_ERR_SHAPE, "grid too small");
    WTD_REQUIRE(sys->cell[0] > 0 && sys->cell[1] > 0 && sys->cell[2] > 0, WTD_ERR_ARG,
                "cell lengths must be positive");
    WTD_REQUIRE(sys->prec == WTD_FP64 || sys->prec == WTD_FP32, WTD_ERR_ARG, "bad precision");
    WTD_REQUIRE((sys->term_mask & ~31u) == 0, WTD_ERR_ARG, "bad term mask");
    WTD_REQUIRE(std::isfinite(sys->alpha) && std::isfinite(sys->k1e_scale) &&
                    std::isfinite(sys->v_g0),
                WTD_ERR_ARG, "non-finite scalar parameter");
    std::unique_ptr<wtd_ctx> c(new wtd_ctx());
    c->stream = (hipStream_t)hip_stream;
    WTD_HIP(hipGetDevice(&c->device));
    c->scratch = scratch_address(c->device);
    c->prec = sys->prec;
    c->mask = sys->term_mask;
    c->npw = sys->npw;
    c->nocc = sys->nocc;
    c->nc = sys->ncond;
    c->max_nb = max_nb;
    c->alpha = sys->alpha;
    c->ck = sys->k1e_scale;
    c->vg0 = sys->v_g0;
    c->eps_occ_h.assign(sys->eps_occ, sys->eps_occ + sys->nocc);
    c->eps_cond_h.assign(sys->eps_cond, sys->eps_cond + sys->ncond);
    try {
      if (c->prec == WTD_FP64) {
        create_impl<double>(c.get(), sys);
        transform_occ<double>(c.get(), sys->c_occ);
      } else {
        create_impl<float>(c.get(), sys);
        transform_occ<float>(c.get(), sys->c_occ);
      }
      WTD_HIP(hipStreamSynchronize(c->stream));
    } catch (...) {
      free_all(c.get());
      throw;
    }
    *out = c.release();
    return WTD_OK;
  });
}

wtd_status wtd_destroy(wtd_ctx* ctx) {
  if (!ctx) return WTD_OK;
  return guarded([&]() -> wtd_status {
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return WTD_OK;
  });
}

wtd_status wtd_set_occ(wtd_ctx* ctx, const double* c_occ) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && c_occ, WTD_ERR_ARG, "null argument");
    if (ctx->checks & WTD_CHECK_FINITE)
      require_finite<double>(ctx, c_occ, (int64_t)ctx->nocc * 2 * ctx->npw, "c_occ");
    ctx->tau_valid = false;
    if (ctx->prec == WTD_FP64)
      transform_occ<double>(ctx, c_occ);
    else
      transform_occ<float>(ctx, c_occ);
    return WTD_OK;
  });
}

wtd_status wtd_cache_pairs(wtd_ctx* ctx, int32_t on) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx, WTD_ERR_ARG, "null context");
    WTD_REQUIRE(!on || ctx->row_block == 0 || ctx->bpairs.size() == 1, WTD_ERR_SHAPE,
                "the row-blocked exchange keeps the pair potentials of one block pair only");
    ctx->tau_cache = on != 0;
    ctx->tau_valid = false;
    return WTD_OK;
  });
}

wtd_status wtd_autotune(wtd_ctx* ctx, int32_t nb, int32_t reps, int32_t* chunk,
                        int32_t* groups) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx, WTD_ERR_ARG, "null context");
    WTD_REQUIRE(nb >= 1 && nb <= ctx->max_nb, WTD_ERR_SHAPE, "nb out of range [1, max_nb]");
    WTD_REQUIRE(reps >= 1 && reps <= 100, WTD_ERR_ARG, "reps out of range [1, 100]");
    if (ctx->prec == WTD_FP64)
      autotune_impl<double>(ctx, nb, reps, chunk, groups);
    else
      autotune_impl<float>(ctx, nb, reps, chunk, groups);
    return WTD_OK;
  });
}

wtd_status wtd_apply_liouville(wtd_ctx* ctx, int32_t nb, const void* a, void* la) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && a && la, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nb >= 1 && nb <= ctx->max_nb, WTD_ERR_SHAPE, "nb out of range [1, max_nb]");
    WTD_REQUIRE(a != la, WTD_ERR_ARG, "a and la must not alias");
    const int64_t len = (int64_t)nb * ctx->nocc * 2 * ctx->npw;
    const bool chk = ctx->checks & WTD_CHECK_FINITE;
    if (chk) require_finite_any(ctx, a, len, "the trial block a");
    if (ctx->prec == WTD_FP64)
      apply_impl<double>(ctx, nb, (const double*)a, (double*)la, tda_mask(ctx));
    else
      apply_impl<float>(ctx, nb, (const float*)a, (float*)la, tda_mask(ctx));
    if (chk) require_finite_any(ctx, la, len, "the result la");
    return WTD_OK;
  });
}

wtd_status wtd_apply_full(wtd_ctx* ctx, int32_t nb, const void* a, void* la) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && a && la, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nb >= 1 && nb <= ctx->max_nb, WTD_ERR_SHAPE, "nb out of range [1, max_nb]");
    WTD_REQUIRE(a != la, WTD_ERR_ARG, "a and la must not alias");
    const int64_t len = (int64_t)nb * ctx->nocc * 2 * ctx->npw;
    const bool chk = ctx->checks & WTD_CHECK_FINITE;
    if (chk) require_finite_any(ctx, a, len, "the trial block a");
    if (ctx->prec == WTD_FP64)
      apply_impl<double>(ctx, nb, (const double*)a, (double*)la, ctx->mask);
    else
      apply_impl<float>(ctx, nb, (const float*)a, (float*)la, ctx->mask);
    if (chk) require_finite_any(ctx, la, len, "the result la");
    return WTD_OK;
  });
}

wtd_status wtd_solve_zvector(wtd_ctx* ctx, int32_t nrhs, const double* U, double tol,
                             int32_t max_iter, double lambda_thr, double* Z, double* resid,
                             int32_t* n_iter, int32_t* n_exact) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && U && Z, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nrhs >= 1 && nrhs <= ctx->max_nb, WTD_ERR_SHAPE, "nrhs out of range [1, max_nb]");
    WTD_REQUIRE(max_iter >= 1 && tol > 0.0 && lambda_thr >= 0.0, WTD_ERR_ARG,
                "need max_iter >= 1, tol > 0 and lambda_thr >= 0");
    WTD_REQUIRE((const void*)U != (void*)Z, WTD_ERR_ARG, "U and Z must not alias");
    return zvector_impl(ctx, nrhs, U, tol, max_iter, lambda_thr, Z, resid, n_iter, n_exact);
  });
}

wtd_status wtd_apply_transition(wtd_ctx* ctx, int32_t nb, const double* X, double* T) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && X && T, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nb >= 1 && nb <= ctx->max_nb, WTD_ERR_SHAPE, "nb out of range [1, max_nb]");
    WTD_REQUIRE((const void*)X != (void*)T, WTD_ERR_ARG, "X and T must not alias");
    const int64_t len = (int64_t)nb * ctx->nocc * ctx->nc;
    const bool chk = ctx->checks & WTD_CHECK_FINITE;
    if (chk) require_finite<double>(ctx, X, len, "the transition block X");
    apply_transition_any(ctx, nb, X, T, tda_mask(ctx));
    if (chk) require_finite<double>(ctx, T, len, "the result T");
    return WTD_OK;
  });
}

wtd_status wtd_apply_liouville_bwd(wtd_ctx* ctx, int32_t nb, const void* a, const void* g_la,
                                   void* g_a, void* g_occ) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && a && g_la, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nb >= 1 && nb <= ctx->max_nb, WTD_ERR_SHAPE, "nb out of range [1, max_nb]");
    WTD_REQUIRE(nb <= 16, WTD_ERR_SHAPE, "the backward apply takes at most 16 trials per call");
    WTD_REQUIRE(g_a != a && g_a != g_la && g_occ != a && g_occ != g_la, WTD_ERR_ARG,
                "outputs must not alias the inputs");
    if (ctx->checks & WTD_CHECK_FINITE) {
      const int64_t len = (int64_t)nb * ctx->nocc * 2 * ctx->npw;
      require_finite_any(ctx, a, len, "the trial block a");
      require_finite_any(ctx, g_la, len, "the cotangent g_la");
    }
    if (ctx->prec == WTD_FP64)
      bwd_impl<double>(ctx, nb, (const double*)a, (const double*)g_la, (double*)g_a,
                       (double*)g_occ);
    else
      bwd_impl<float>(ctx, nb, (const float*)a, (const float*)g_la, (float*)g_a, (float*)g_occ);
    return WTD_OK;
  });
}

wtd_status wtd_davidson(wtd_ctx* ctx, int32_t nroots, int32_t nb, double tol, int32_t max_iter,
                        int32_t max_sub, const double* guess, double* omega, double* x,
                        double* resid, int32_t* n_iter) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && omega, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nroots >= 1 && nb >= nroots && nb <= ctx->max_nb, WTD_ERR_SHAPE,
                "need 1 <= nroots <= nb <= max_nb");
    WTD_REQUIRE(max_iter >= 1 && tol > 0.0, WTD_ERR_ARG, "need max_iter >= 1 and tol > 0");
    return davidson_impl(ctx, nroots, nb, tol, max_iter, max_sub, guess, omega, x, resid,
                         n_iter);
  });
}

wtd_status wtd_davidson_noalloc(wtd_ctx* ctx, int32_t nroots, int32_t nb, double tol,
                                int32_t max_iter, int32_t max_sub, const double* guess,
                                double* omega, double* x, double* resid, int32_t* n_iter) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx && omega, WTD_ERR_ARG, "null argument");
    WTD_REQUIRE(nroots >= 1 && nb >= nroots && nb <= ctx->max_nb, WTD_ERR_SHAPE,
                "need 1 <= nroots <= nb <= max_nb");
    WTD_REQUIRE(max_iter >= 1 && tol > 0.0, WTD_ERR_ARG, "need max_iter >= 1 and tol > 0");
    return davidson_impl(ctx, nroots, nb, tol, max_iter, max_sub, guess, omega, x, resid,
                         n_iter, true);
  });
}

wtd_status wtd_profile_enable(wtd_ctx* ctx, int32_t on) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx, WTD_ERR_ARG, "null context");
    if (!on) prof_collect(ctx);
    ctx->prof.on = on != 0;
    return WTD_OK;
  });
}

wtd_status wtd_profile_read(wtd_ctx* ctx, int32_t n, double* ms, int64_t* calls,
                            const char** names, int32_t* count) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx, WTD_ERR_ARG, "null context");
    Profiler& P = ctx->prof;
    prof_collect(ctx);
    for (int i = 0; i < std::min<int>(n, Profiler::kStages); ++i) {
      if (ms) ms[i] = P.ms[i];
      if (calls) calls[i] = P.calls[i];
      if (names) names[i] = P.names[i];
      P.ms[i] = 0.0;
      P.calls[i] = 0;
    }
    if (count) *count = Profiler::kStages;
    return WTD_OK;
  });
}

wtd_status wtd_set_workspace_limit(size_t bytes) {
  g_workspace_limit.store(bytes);
  return WTD_OK;
}

wtd_status wtd_set_checks(wtd_ctx* ctx, uint32_t flags) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(ctx, WTD_ERR_ARG, "null context");
    WTD_REQUIRE((flags & ~(uint32_t)WTD_CHECK_FINITE) == 0, WTD_ERR_ARG, "unknown check flag");
    ctx->checks = flags;
    return WTD_OK;
  });
}

wtd_status wtd_workspace_bytes(const wtd_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) {
    set_error("null argument");
    return WTD_ERR_ARG;
  }
  *bytes = ctx->total_bytes;
  return WTD_OK;
}

}  // extern "C"

#include "../../include/wtd_debug.h"

extern "C" wtd_status wtd_debug_gemm(wtd_precision prec, int32_t m, int32_t n, int32_t k,
                                     const void* a, int32_t lda, const void* b, int32_t ldb,
                                     int32_t b_kmajor, void* c, int32_t ldc, void* hip_stream) {
  return guarded([&]() -> wtd_status {
    WTD_REQUIRE(a && b && c && m >= 0 && n >= 0 && k >= 0, WTD_ERR_ARG, "bad GEMM arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    if (prec == WTD_FP64) {
      if (b_kmajor)
        launch_gemm<double, true>(m, n, k, (const double*)a, lda, (const double*)b, ldb,
                                  (double*)c, ldc, s);
      else
        launch_gemm<double, false>(m, n, k, (const double*)a, lda, (const double*)b, ldb,
                                   (double*)c, ldc, s);
    } else {
      if (b_kmajor)
        launch_gemm<float, true>(m, n, k, (const float*)a, lda, (const float*)b, ldb, (float*)c,
                                 ldc, s);
      else
        launch_gemm<float, false>(m, n, k, (const float*)a, lda, (const float*)b, ldb, (float*)c,
                                  ldc, s);
    }
    return WTD_OK;
  });
}
