// FP64 kernels of the block Davidson solver (the paper's Sec. 4 diagonalises
// the Liouville super-operator with the Davidson method; the normalisation
// sum_v <a_v|a_v> = 1 is the constraint of Eq. ltda).
//
// Vectors live in transition coordinates X[v][c] (length n = Nocc Nc), stored
// as rows of row-major matrices.  All reductions are deterministic
// (fixed-order tree sums, no atomics).
#include "wtd_internal.h"

namespace wtd {

namespace {

constexpr int kRed = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// out[i*ldo + j] = A_i . B_j
__global__ void __launch_bounds__(kRed)
k_gram(const double* __restrict__ A, const double* __restrict__ B, int64_t n,
       double* __restrict__ out, int ldo) {
  __shared__ double sh[kRed];
  const int i = blockIdx.x, j = blockIdx.y;
  const double* a = A + (int64_t)i * n;
  const double* b = B + (int64_t)j * n;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += a[r] * b[r];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[(int64_t)i * ldo + j] = s;
}

// out[j][r] = sum_i V[i][r] Y[i*ldy + j]
__global__ void k_lincomb(const double* __restrict__ V, int m, int64_t n,
                          const double* __restrict__ Y, int ldy, int k, double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= n || j >= k) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += V[(int64_t)i * n + r] * Y[(int64_t)i * ldy + j];
  out[(int64_t)j * n + r] = s;
}

// R_j = WY_j - theta_j X_j ; rnorm2[j] = |R_j|^2
__global__ void __launch_bounds__(kRed)
k_residual(const double* __restrict__ WY, const double* __restrict__ X,
           const double* __restrict__ theta, int64_t n, double* __restrict__ R,
           double* __restrict__ rnorm2) {
  __shared__ double sh[kRed];
  const int j = blockIdx.x;
  const double th = theta[j];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double v = WY[(int64_t)j * n + r] - th * X[(int64_t)j * n + r];
    R[(int64_t)j * n + r] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) rnorm2[j] = s;
}

// T_j = R_{active[j]} / (diag - theta_{active[j]}), denominator magnitude floored at 1e-3
__global__ void k_precondition(const double* __restrict__ R, const double* __restrict__ theta,
                               const double* __restrict__ diag, int64_t n,
                               const int* __restrict__ active, double* __restrict__ T) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= n) return;
  const int src = active[j];
  double den = diag[r] - theta[src];
  if (fabs(den) < 1e-3) den = den < 0.0 ? -1e-3 : 1e-3;
  T[(int64_t)j * n + r] = R[(int64_t)src * n + r] / den;
}

// t_j -= sum_i coef[i*k + j] V_i
__global__ void k_axpy_cols(double* __restrict__ t, const double* __restrict__ V,
                            const double* __restrict__ coef, int m, int k, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= n) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += coef[(int64_t)i * k + j] * V[(int64_t)i * n + r];
  t[(int64_t)j * n + r] -= s;
}

__global__ void __launch_bounds__(kRed)
k_row_norm2(const double* __restrict__ t, int64_t n, double* __restrict__ out) {
  __shared__ double sh[kRed];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double v = t[(int64_t)j * n + r];
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = s;
}

__global__ void __launch_bounds__(kRed)
k_row_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
          double* __restrict__ out) {
  __shared__ double sh[kRed];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x)
    s += a[(int64_t)j * n + r] * b[(int64_t)j * n + r];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// conjugate-gradient updates of k independent systems, step sizes per row:
// z_j += alpha_j p_j, r_j -= alpha_j Ap_j
__global__ void k_cg_update(double* __restrict__ z, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ ap,
                            const double* __restrict__ alpha, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const int64_t o = (int64_t)j * n + i;
  const double a = alpha[j];
  z[o] += a * p[o];
  r[o] -= a * ap[o];
}

// p_j = r_j + beta_j p_j
__global__ void k_cg_direction(double* __restrict__ p, const double* __restrict__ r,
                               const double* __restrict__ beta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const int64_t o = (int64_t)j * n + i;
  p[o] = r[o] + beta[j] * p[o];
}

__global__ void k_scale_row(double* __restrict__ t, double f, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) t[r] *= f;
}

// Cyclic parallel Jacobi for a symmetric m x m matrix (one workgroup).
// H (ld) is symmetrised on entry and destroyed.  evals ascending, evecs[i*m + j]
// is component i of eigenvector j.  Round-robin (circle) pairing: in round r
// the pairs are (r mod (mm-1), mm-1) and ((r+k) mod (mm-1), (r-k) mod (mm-1)),
// k = 1..mm/2-1, with mm = m rounded up to even; indices >= m are skipped.
// Rotation of a pair (p, q): tau = (a_qq - a_pp)/(2 a_pq),
// t = sign(tau)/(|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c;
// A <- J^T A J with J_pp = J_qq = c, J_pq = s, J_qp = -s (Golub & Van Loan).
__global__ void __launch_bounds__(256)
k_jacobi(double* __restrict__ A, int m, int ld, double* __restrict__ Vv,
         double* __restrict__ evals, double* __restrict__ evecs) {
  __shared__ double cs_c[128], cs_s[128];
  __shared__ int pp[128], qq[128];
  __shared__ double red[256];
  __shared__ int perm[256];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < m * m; e += nt) Vv[e] = (e / m == e % m) ? 1.0 : 0.0;
  // symmetrised compact (leading dimension m) copy of H, staged through evecs
  for (int e = tid; e < m * m; e += nt) {
    const int i = e / m, j = e % m;
    evecs[e] = 0.5 * (A[(int64_t)i * ld + j] + A[(int64_t)j * ld + i]);
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += nt) A[e] = evecs[e];
  __syncthreads();
  const int mm = (m + 1) & ~1;
  const int npair = mm / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // off-diagonal and total norms
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e % m;
      const double a = A[e];
      tot += a * a;
      if (i != j) off += a * a;
    }
    red[tid] = off;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    off = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    tot = red[0];
    __syncthreads();
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int r = 0; r < mm - 1; ++r) {
      for (int k = tid; k < npair; k += nt) {
        int p, q;
        if (k == 0) {
          p = r % (mm - 1);
          q = mm - 1;
        } else {
          p = (r + k) % (mm - 1);
          q = (r - k + (mm - 1)) % (mm - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[p * m + q];
          if (apq != 0.0) {
            const double app = A[p * m + p], aqq = A[q * m + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[k] = p; qq[k] = q; cs_c[k] = c; cs_s[k] = s;
      }
      __syncthreads();
      // rows: A[p][j], A[q][j]
      for (int e = tid; e < npair * m; e += nt) {
        const int k = e / m, j = e % m;
        const int p = pp[k], q = qq[k];
        if (q >= m || cs_s[k] == 0.0) continue;
        const double c = cs_c[k], s = cs_s[k];
        const double ap = A[p * m + j], aq = A[q * m + j];
        A[p * m + j] = c * ap - s * aq;
        A[q * m + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns of A and of the eigenvector matrix
      for (int e = tid; e < npair * m; e += nt) {
        const int k = e / m, i = e % m;
        const int p = pp[k], q = qq[k];
        if (q >= m || cs_s[k] == 0.0) continue;
        const double c = cs_c[k], s = cs_s[k];
        const double ap = A[i * m + p], aq = A[i * m + q];
        A[i * m + p] = c * ap - s * aq;
        A[i * m + q] = s * ap + c * aq;
        const double vp = Vv[i * m + p], vq = Vv[i * m + q];
        Vv[i * m + p] = c * vp - s * vq;
        Vv[i * m + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // ascending order by rank (ties broken by index)
  for (int j = tid; j < m; j += nt) {
    const double dj = A[j * m + j];
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      const double di = A[i * m + i];
      if (di < dj || (di == dj && i < j)) ++rank;
    }
    perm[rank] = j;
  }
  __syncthreads();
  for (int j = tid; j < m; j += nt) evals[j] = A[perm[j] * m + perm[j]];
  for (int e = tid; e < m * m; e += nt) {
    const int i = e / m, j = e % m;
    evecs[e] = Vv[i * m + perm[j]];
  }
}

// indices j < k with rnorm2[j] > tol2, in order (the roots that still get a
// correction; the host applies the same test to the same values); one thread
__global__ void k_active_list(const double* __restrict__ rnorm2, int k, double tol2,
                              int* __restrict__ active) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int c = 0;
  for (int j = 0; j < k; ++j)
    if (rnorm2[j] > tol2) active[c++] = j;
}

__global__ void k_sub_rows(double* __restrict__ t, const double* __restrict__ d, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) t[i] -= d[i];
}

// Normalise row t (length n) or, if its norm is below 1e-10 (the correction
// lies in the span of the basis), zero it; ok[slot] records which.
__global__ void __launch_bounds__(kRed)
k_normalise_or_drop(double* __restrict__ t, int64_t n, int* __restrict__ ok, int slot) {
  __shared__ double sh[kRed];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += t[r] * t[r];
  s = block_sum(s, sh);
  const double nrm = sqrt(s);
  const bool keep = nrm >= 1e-10;
  const double f = keep ? 1.0 / nrm : 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) t[r] *= f;
  if (threadIdx.x == 0) ok[slot] = keep ? 1 : 0;
}

// Basis slots holding a dropped (zero) correction have zero rows and columns
// in the subspace matrix; their diagonal is set to 2 g + 1, g the largest
// absolute row sum of the kept slots (a Gershgorin bound on its eigenvalues),
// so their Ritz values sort after every Ritz value of the kept basis without
// changing the scale of the matrix.  One workgroup.
__global__ void __launch_bounds__(kRed)
k_fix_dropped(double* __restrict__ H, int ld, const int* __restrict__ ok, int m) {
  __shared__ double sh[kRed];
  double g = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    if (!ok[i]) continue;
    double r = 0.0;
    for (int j = 0; j < m; ++j) r += fabs(H[(int64_t)i * ld + j]);
    g = fmax(g, r);
  }
  sh[threadIdx.x] = g;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  const double big = 2.0 * sh[0] + 1.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x)
    if (!ok[i]) H[(int64_t)i * ld + i] = big;
}

// out[j][i] = in[i][j] for an r x c row-major matrix
__global__ void k_transpose(const double* __restrict__ in, int r, int c, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * c) return;
  const int i = e / c, j = e % c;
  out[(int64_t)j * r + i] = in[e];
}

dim3 rows_grid(int64_t n, int k) { return dim3((unsigned)((n + 255) / 256), (unsigned)k); }

}  // namespace

void launch_gram(const double* A, int na, const double* B, int nbv, int64_t n, double* out,
                 int ldo, hipStream_t s) {
  if (na <= 0 || nbv <= 0) return;
  hipLaunchKernelGGL(k_gram, dim3(na, nbv), dim3(kRed), 0, s, A, B, n, out, ldo);
  WTD_HIP(hipGetLastError());
}

void launch_lincomb(const double* V, int m, int64_t n, const double* Y, int ldy, int k,
                    double* out, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_lincomb, rows_grid(n, k), dim3(256), 0, s, V, m, n, Y, ldy, k, out);
  WTD_HIP(hipGetLastError());
}

void launch_residual(const double* WY, const double* X, const double* theta, int k, int64_t n,
                     double* R, double* rnorm2, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_residual, dim3(k), dim3(kRed), 0, s, WY, X, theta, n, R, rnorm2);
  WTD_HIP(hipGetLastError());
}

void launch_precondition(const double* R, const double* theta, const double* diag, int k,
                         int64_t n, const int* active, double* T, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_precondition, rows_grid(n, k), dim3(256), 0, s, R, theta, diag, n,
                     active, T);
  WTD_HIP(hipGetLastError());
}

void launch_jacobi_eig(double* H, int m, int ld, double* evals, double* evecs, hipStream_t s) {
  // evecs must hold m*m doubles; H must hold max(ld*m, m*m) doubles and is
  // reused as compact scratch; a second m*m scratch follows evecs' partner below.
  WTD_REQUIRE(m >= 1 && m <= 256, WTD_ERR_SHAPE, "subspace dimension out of range");
  double* Vv = evecs + (int64_t)m * m;  // caller provides 2*m*m doubles at evecs
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), 0, s, H, m, ld, Vv, evals, evecs);
  WTD_HIP(hipGetLastError());
}

void launch_axpy_cols(double* t, const double* V, const double* coef, int m, int k, int64_t n,
                      hipStream_t s) {
  if (k <= 0 || m <= 0) return;
  hipLaunchKernelGGL(k_axpy_cols, rows_grid(n, k), dim3(256), 0, s, t, V, coef, m, k, n);
  WTD_HIP(hipGetLastError());
}

void launch_col_norms(const double* t, int k, int64_t n, double* out, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_row_norm2, dim3(k), dim3(kRed), 0, s, t, n, out);
  WTD_HIP(hipGetLastError());
}

void launch_col_dots(const double* a, const double* b, int k, int64_t n, double* out,
                     hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_row_dot, dim3(k), dim3(kRed), 0, s, a, b, n, out);
  WTD_HIP(hipGetLastError());
}

void launch_cg_update(double* z, double* r, const double* p, const double* ap,
                      const double* alpha, int k, int64_t n, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_cg_update, rows_grid(n, k), dim3(256), 0, s, z, r, p, ap, alpha, n);
  WTD_HIP(hipGetLastError());
}

void launch_cg_direction(double* p, const double* r, const double* beta, int k, int64_t n,
                         hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_cg_direction, rows_grid(n, k), dim3(256), 0, s, p, r, beta, n);
  WTD_HIP(hipGetLastError());
}

void launch_scale_rows(double* t, double f, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_row, rows_grid(n, 1), dim3(256), 0, s, t, f, n);
  WTD_HIP(hipGetLastError());
}

void launch_active_list(const double* rnorm2, int k, double tol2, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_active_list, dim3(1), dim3(64), 0, s, rnorm2, k, tol2, active);
  WTD_HIP(hipGetLastError());
}

void launch_sub_rows(double* t, const double* d, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_sub_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, t, d,
                     total);
  WTD_HIP(hipGetLastError());
}

void launch_normalise_or_drop(double* t, int64_t n, int* ok, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_normalise_or_drop, dim3(1), dim3(kRed), 0, s, t, n, ok, slot);
  WTD_HIP(hipGetLastError());
}

void launch_fix_dropped(double* H, int ld, const int* ok, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_fix_dropped, dim3(1), dim3(kRed), 0, s, H, ld, ok, m);
  WTD_HIP(hipGetLastError());
}

void launch_transpose(const double* in, int r, int c, double* out, hipStream_t s) {
  if (r * c <= 0) return;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((r * c + 255) / 256)), dim3(256), 0, s, in, r, c,
                     out);
  WTD_HIP(hipGetLastError());
}

}  // namespace wtd
