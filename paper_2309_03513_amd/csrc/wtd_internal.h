// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wtd.h"
#include "wtd_fft.h"

namespace wtd {

void set_error(const std::string& msg);

struct StatusError {
  wtd_status code;
  std::string msg;
};

#define WTD_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::wtd::StatusError{WTD_ERR_HIP, std::string(#call) + ": " +                \
                                                hipGetErrorString(e_)};                \
  } while (0)

#define WTD_REQUIRE(cond, code, msg)                                \
  do {                                                              \
    if (!(cond)) throw ::wtd::StatusError{(code), std::string(msg)}; \
  } while (0)

// ----------------------------------------------------------------------------
// Transform geometry shared by every kernel of one context.
struct Geometry {
  int n0, n1, n2;
  int64_t nr;      // n0*n1*n2
  int plane;       // n1*n2
  double omega;
  FFTPlan plan0, plan1, plan2;
  // plan1 with the column cut of the density sticks and of the wave sticks
  // (the column pass of the compile-time plane kernels; see FFTPlan::cut)
  FFTPlan plan1d, plan1w;
  // twiddle tables (one per axis), device, working precision
  const void* tw0;
  const void* tw1;
  const void* tw2;
  // wave sticks: columns along i0 of the wave-function sphere
  int nw;                 // number of wave sticks
  int nws;                // stick row stride of wave-stick buffers (nw rounded up to 16)
  const int* wst_k12;     // [nw] k1*n2 + k2
  int nwtile;             // stick tiles for the sphere->stick scatter
  const int* wtile_off;   // [nwtile+1] CSR offsets into wtile_ent
  const int4* wtile_ent;  // entries (h, sign, local stick, k0)
  const int2* sph_pos;    // [npw] (stick*n0 + k0) of +m and of -m
  // density sticks: columns that pair products can occupy
  int nd;
  int nds;                // stick row stride of density-stick buffers (nd rounded up to 16)
  const int* dst_k12;     // [nd]
  const void* dkern;      // [nd][n0] Coulomb kernel / N_r, working precision
  // rows k1 of the density and wave stick sets: (k1, first stick, R, 0), the
  // row holding k2 = 0..R and n2 - R..n2 - 1 (0 rows: not of that form)
  int ndrow, nwrow;
  const int4* drows;
  const int4* wrows;
  // plane size of the register-quad plane kernels, used where the complex plane
  // does not fit in LDS (0: the LDS plane kernels)
  int quad_sn;
};

constexpr int kStickTile = 16;

// ----------------------------------------------------------------------------
// Kernel launchers (wtd_transforms.hip)
// compile-time plane size of the wave-stick plane kernels (0: runtime plans)
int plane_static_wave(const Geometry& g);
// plane size for the register-quad plane kernels of a context of element size
// `elem` (0: none); force takes them wherever they apply (a test hook)
int quad_plane_size(const Geometry& g, size_t elem, bool force);
template <typename T>
void launch_sphere_to_wsticks(const Geometry& g, const T* coef, int nfield, int npw, int nb,
                              int per_trial, cplx<T>* wst, hipStream_t s);
// With drho and a partial buffer part [ngroup][nb][nr], the orbital loop of each
// trial is split over ngroup workgroups and the partial densities are summed.
template <typename T>
void launch_wsticks_to_fields(const Geometry& g, const cplx<T>* wst, int nb, int per_trial,
                              int nfield_per_trial, T scale, T* out, const T* phi,
                              T* drho, hipStream_t s, T* part = nullptr, int ngroup = 1);
template <typename T>
void launch_pairs_to_dsticks(const Geometry& g, const T* src, const int4* quads, int npack,
                             int limit, cplx<T>* dst, hipStream_t s);
template <typename T>
void launch_dstick_poisson(const Geometry& g, cplx<T>* dst, int npack, hipStream_t s);
// Pair potentials read by the round-robin contraction are stored interleaved by
// groups of kTauIl pairs: pair P at point r is element ((P / kTauIl) N_r + r) kTauIl + P % kTauIl.
constexpr int kTauIl = 4;
constexpr int kTauIlShift = 2;
static_assert((1 << kTauIlShift) == kTauIl, "interleave factor is a power of two");

// il: write fields into the interleaved layout above
template <typename T>
void launch_dsticks_to_fields(const Geometry& g, const cplx<T>* dst, int npack, int nfield,
                              T* out, hipStream_t s, bool il = false);
// K2d inverse pass fused with its contraction (72 x 72 planes, even Nocc):
// dst holds packs p = j (nocc / 2) + k for rows j < nrows of the chunk starting
// at row r0; R (one trial) -= alpha sum_v' phi_v' W_v'v.  Returns false where it
// does not apply (the caller then writes W and runs launch_k2d_rows).
bool k2d_inverse_applies(const Geometry& g, int nocc);
template <typename T>
bool launch_k2d_inverse(const Geometry& g, const cplx<T>* dst, int nrows, int r0, int nocc,
                        const T* phi, T alpha, T* R, hipStream_t s);
template <typename T>
void launch_fields_to_wsticks(const Geometry& g, const T* fields, int nb, int per_trial,
                              int nfield_per_trial, cplx<T>* wst, hipStream_t s);
template <typename T>
void launch_wsticks_to_sphere(const Geometry& g, cplx<T>* wst, int npack, hipStream_t s);
template <typename T>
void launch_extract_sphere(const Geometry& g, const cplx<T>* wst, int nb, int per_trial,
                           int nfield_per_trial, int npw, T scale, T* coef, hipStream_t s);
template <typename T>
void launch_contract(const Geometry& g, int nb, int nocc, const T* phi, const T* at,
                     const T* tau, const int* pair_index, const T* vh, const T* drho,
                     const T* fxc, T ck, T alpha, bool k1e, bool k1d, T* R, hipStream_t s);

// Pair order of the round-robin contraction (FP32, Nocc = 128, all pairs at
// once): the 36 tiles (I <= J) of 16 x 16 occupied rows in row-major tile
// order; a diagonal tile holds its upper triangle row by row (136 pairs, the
// pair (16 I + a, 16 I + b), a <= b, at rr_tri_index(a, b)), an off-diagonal
// tile its full square row-major (256 pairs).  Both counts are multiples of
// kTauIl, so every tile starts on a whole interleave group.
__host__ __device__ constexpr int rr_tile_base(int I, int J) {
  return 136 * I + 256 * (7 * I - I * (I - 1) / 2) + (J > I ? 136 + 256 * (J - I - 1) : 0);
}
__host__ __device__ constexpr int rr_tri_index(int a, int b) {
  return 16 * a - a * (a - 1) / 2 + (b - a);
}

// MFMA contraction for Nocc <= 128 (wtd_contract.hip); returns false if not applicable.
// tau is [pair][N_r] (pairs v <= v' row-major); with tau_il set (only where
// contract_rr_applies(): FP32, Nocc = 128, N_r a multiple of 8, any nb) it
// holds the pairs in the tile order above, in the kTauIl-interleaved layout
// read by the round-robin kernel.
template <typename T>
bool contract_rr_applies(const Geometry& g, int nb, int nocc);
template <typename T>
bool launch_contract_mfma(const Geometry& g, int nb, int nocc, const T* phi, const T* at,
                          const T* tau, const T* vh, const T* drho, const T* fxc, T ck, T alpha,
                          bool k1e, bool k1d, T* R, hipStream_t s, bool tau_il);

// Block form of the exchange contraction for large Nocc (wtd_contract.hip):
// R = c_K phi (v_H + f_xc drho) first, then per row block pair (A, B)
// R[A] -= alpha tau a[B] and R[B] -= alpha tau^T a[A] (tau of the block only).
template <typename T>
void launch_response_rows(const Geometry& g, int nb, int nocc, const T* phi, const T* vh,
                          const T* drho, const T* fxc, T ck, bool k1e, T* R, hipStream_t s);
template <typename T>
void launch_contract_block(const Geometry& g, int nb, int nocc, const T* at, const T* tau, int A0,
                           int nA, int B0, int nB, bool diag, T alpha, T* R, hipStream_t s);

// The same with tau in the kTauIl-interleaved layout (FP32): one pass over the
// block's tau for 32 trials at a time (trials past nb are zero).
template <typename T>
bool contract_block_rr_applies(int nb);
template <typename T>
void launch_contract_block_rr(const Geometry& g, int nb, int nocc, const T* at, const T* tau,
                              int A0, int nA, int B0, int nB, bool diag, T alpha, T* R,
                              hipStream_t s);

// K2d contraction of one trial (wtd_contract.hip): for rows v' in [r0, r0 + nrows),
// R[v] -= alpha sum_v' phi_v' W[(v' - r0) nocc + v], W the Poisson-solved products
// a_v' phi_v stored [pair][N_r].
template <typename T>
void launch_k2d_rows(const Geometry& g, int nocc, int nrows, int r0, const T* phi, const T* W,
                     T alpha, T* R, hipStream_t s);

// Backward kernels (wtd_backward.hip).
// Pair densities of rows [A0, A0 + nA) x [B0, B0 + nB) (diag: the upper
// triangle of one block), stored in the block layout of the pair pipeline.
template <typename T>
void launch_pair_density(const Geometry& g, int nb, int nocc, const T* X, const T* Y, int A0,
                         int nA, int B0, int nB, bool diag, T* P, hipStream_t s);
template <typename T>
void launch_gamma_k1e(const Geometry& g, int nb, int nocc, T ck, const T* gt, const T* at,
                      const T* vh, const T* drho, const T* vhg, const T* drhog, const T* fxc,
                      T* gamma, hipStream_t s);
// mode 0: divide by the half-sphere weights, mode 1: multiply; Im at m = 0 zeroed
template <typename T>
void launch_weights(T* x, int64_t nf, int npw, int mode, hipStream_t s);

// GEMMs (wtd_gemm.hip).  C[m][n] = sum_k A[m*lda + k] * B(k, n), with
// B(k, n) = B[n*ldb + k] (B_KMAJOR) or B[k*ldb + n].
// With a scratch buffer, short-and-wide problems split K into slices whose
// partial products are summed in a fixed order.
template <typename T, bool B_KMAJOR>
void launch_gemm(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                 hipStream_t s, T* scratch = nullptr, size_t scratch_elems = 0);

// Small elementwise kernels (wtd_transforms.hip)
template <typename T>
void launch_dterm_combine(int nb, int nocc, int nc, const T* S, const T* Q, const double* eps_occ,
                          const double* eps_cond, bool with_d, T* out, hipStream_t s);
template <typename Tin, typename Tout>
void launch_convert(const Tin* in, Tout* out, int64_t n, hipStream_t s);
template <typename T>
void launch_zero(T* p, int64_t n, hipStream_t s);
// *flag |= 1 if x[0..n) holds a NaN or an infinity
template <typename T>
void launch_flag_nonfinite(const T* x, int64_t n, unsigned* flag, hipStream_t s);
void launch_transition_out(int nb, int nocc, int nc, const void* Q, bool q_is_float,
                           const double* X, const double* eps_occ, const double* eps_cond,
                           bool with_d, double* T, hipStream_t s);

// Davidson helpers (wtd_davidson.hip), FP64
void launch_gram(const double* A, int na, const double* B, int nbv, int64_t n, double* out,
                 int ldo, hipStream_t s);
void launch_lincomb(const double* V, int m, int64_t n, const double* Y, int ldy, int k,
                    double* out, hipStream_t s);
void launch_residual(const double* WY, const double* X, const double* theta, int k, int64_t n,
                     double* R, double* rnorm2, hipStream_t s);
void launch_precondition(const double* R, const double* theta, const double* diag, int k,
                         int64_t n, const int* active, double* T, hipStream_t s);
void launch_jacobi_eig(double* H, int m, int ld, double* evals, double* evecs, hipStream_t s);
void launch_axpy_cols(double* t, const double* V, const double* coef, int m, int k, int64_t n,
                      hipStream_t s);
void launch_col_norms(const double* t, int k, int64_t n, double* out, hipStream_t s);
void launch_scale_rows(double* t, double f, int64_t n, hipStream_t s);
// rows of k x n arrays: out[j] = a_j . b_j; CG steps with per-row coefficients
void launch_col_dots(const double* a, const double* b, int k, int64_t n, double* out,
                     hipStream_t s);
void launch_cg_update(double* z, double* r, const double* p, const double* ap,
                      const double* alpha, int k, int64_t n, hipStream_t s);
void launch_cg_direction(double* p, const double* r, const double* beta, int k, int64_t n,
                         hipStream_t s);
// device-side pieces of one Davidson step (no host synchronisation)
void launch_active_list(const double* rnorm2, int k, double tol2, int* active, hipStream_t s);
void launch_sub_rows(double* t, const double* d, int64_t total, hipStream_t s);
void launch_normalise_or_drop(double* t, int64_t n, int* ok, int slot, hipStream_t s);
void launch_fix_dropped(double* H, int ld, const int* ok, int m, hipStream_t s);
void launch_transpose(const double* in, int r, int c, double* out, hipStream_t s);

}  // namespace wtd
