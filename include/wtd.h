/*
 * wtd.h - C ABI of the MI355X (gfx950) Liouville-apply library for plane-wave,
 * Gamma-point, Tamm-Dancoff hybrid TDDFT.
 *
 * The operator is L = D + K1e - K1d of the paper's Sec. 2.1 (Eqs. dterm,
 * k1eterm, k1d and TDDFT_VEXX_TDA), acting on trial sets A = {a_v} of
 * occupied-orbital-indexed functions (Eq. deltarho with B = 0), projected onto
 * the unoccupied manifold (P_c, defined after Eq. k2dterm).  The eigenproblem
 * is solved with the Davidson method named in Sec. 4.
 *
 * Conventions (Hartree atomic units, v_c = 1/|r - r'|):
 *  - orthorhombic cell L0 x L1 x L2 bohr, Omega = L0 L1 L2; FFT grid n0 x n1 x n2;
 *    a real-space field is stored as f[(i0*n1 + i1)*n2 + i2] (i2 fastest);
 *  - G_m = 2 pi (m0/L0, m1/L1, m2/L2) for Miller indices m;
 *  - a real orbital is phi(r) = Omega^-1/2 sum_{m in S} c(m) e^{i G_m.r} with
 *    c(-m) = conj(c(m)); only the half sphere S+ is passed: m = 0 first, then
 *    every m whose first nonzero component is positive.  Coefficient arrays
 *    are [..][npw][2] (re, im); the imaginary part at m = 0 is ignored;
 *  - inner product <f|g> = sum_{m in S+} w_m Re(conj f_m g_m), w_0 = 1, w_m = 2;
 *  - the unoccupied manifold is the span of the supplied conduction orbitals
 *    (P = sum_c |phi_c><phi_c|) and H_KS acts spectrally on occupied and
 *    conduction orbitals, so D has entries eps_c - eps_v;
 *  - the K1e term carries the spin factor c_K (2: closed-shell singlet; 0: the
 *    spin-flip problem with exchange only, Eq. TDDFT_VEXX_TDA_SF with K1e,SF
 *    dropped); f_xc is a real-space field;
 *  - Coulomb kernel 4 pi/|G|^2 over the whole FFT box, value v_g0 at G = 0.
 *
 * All entry points return a wtd_status; negative values are errors (outputs
 * undefined), positive values are warnings (outputs valid).  wtd_last_error()
 * returns a thread-local message for the last failure.  No exception crosses
 * the ABI.  One context is not thread-safe; distinct contexts are independent.
 * Device pointers are HIP device memory on the device that was current when
 * the context was created; every device operation is ordered on the HIP
 * stream given at creation.  An apply may run its pair potentials on streams
 * of the context's own, forked from that stream after the work already on it
 * and joined back into it before the apply's later stages, so the apply is
 * one stretch of that stream to the caller and to a graph captured on it.
 */
#ifndef WTD_H
#define WTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wtd_ctx wtd_ctx;

typedef enum {
  WTD_OK = 0,
  WTD_NOT_CONVERGED = 1,       /* warning: Davidson stopped at max_iter; outputs valid   */
  WTD_ERR_ARG = -1,            /* null pointer, out-of-range scalar                     */
  WTD_ERR_SHAPE = -2,          /* inconsistent sizes (grid vs sphere, nb > max_nb, ...)  */
  WTD_ERR_OOM = -3,            /* device allocation failed or workspace cap exceeded    */
  WTD_ERR_HIP = -4,            /* a HIP runtime call failed                             */
  WTD_ERR_UNIMPLEMENTED = -5,  /* the requested operation is not provided              */
  WTD_ERR_NONFINITE = -6       /* non-finite values detected (when checking is enabled) */
} wtd_status;

typedef enum { WTD_FP64 = 0, WTD_FP32 = 1 } wtd_precision;

enum { WTD_TERM_D = 1, WTD_TERM_K1E = 2, WTD_TERM_K1D = 4, WTD_TERM_ALL = 7,
       /* the terms of the full operator of the Z-vector equation (Eq. z-v-eq),
        * applied only by wtd_apply_full and wtd_solve_zvector                   */
       WTD_TERM_K2E = 8, WTD_TERM_K2D = 16, WTD_TERM_FULL = 31 };

typedef struct {
  int32_t n[3];            /* FFT grid; each n_i > 2 max|m_i| and n_i a product of 2,3,5   */
  double cell[3];          /* orthorhombic edge lengths (bohr)                              */
  int32_t npw;             /* number of half-sphere plane waves (m = 0 first)               */
  const int32_t *mill;     /* host [npw][3] Miller indices                                  */
  int32_t nocc, ncond;     /* occupied / conduction orbital counts                          */
  const double *c_occ;     /* device [nocc][npw][2] FP64                                     */
  const double *c_cond;    /* device [ncond][npw][2] FP64; orthonormal, orthogonal to c_occ */
  const double *eps_occ;   /* host [nocc] Hartree                                           */
  const double *eps_cond;  /* host [ncond] Hartree                                          */
  const double *fxc;       /* device [n0*n1*n2] Ha bohr^3 (layout above); NULL means 0      */
  double alpha;            /* exact-exchange fraction alpha_EXX                             */
  double k1e_scale;        /* c_K                                                           */
  double v_g0;             /* Coulomb kernel value at G = 0 (0 drops it)                    */
  uint32_t term_mask;      /* WTD_TERM_* subset (WTD_TERM_ALL in production)                */
  wtd_precision prec;      /* FP64, or FP32 bulk arithmetic (transforms, pair potentials,
                              contraction, projections) with FP64 Davidson subspace work    */
} wtd_system;

/* Create a context.  Copies and converts every system array into context-owned
 * device memory (the caller may free its arrays afterwards), transforms the
 * occupied orbitals to real space and allocates the workspace for blocks of up
 * to max_nb trial vectors.  hip_stream is a hipStream_t (NULL: null stream).
 * Errors: WTD_ERR_ARG (null pointers, max_nb < 1, bad term mask / precision),
 * WTD_ERR_SHAPE (grid too small for the sphere, unsupported grid factor,
 * duplicate or out-of-half-space Miller indices, m = 0 not first),
 * WTD_ERR_OOM, WTD_ERR_HIP.  On error *out is set to NULL.                      */
wtd_status wtd_create(const wtd_system *sys, int32_t max_nb, void *hip_stream, wtd_ctx **out);

/* Release every device and host resource of the context (NULL is accepted).    */
wtd_status wtd_destroy(wtd_ctx *ctx);

/* Replace the occupied orbitals (device [nocc][npw][2] FP64, same sphere) and
 * re-transform them to real space.  Asynchronous on the context stream.        */
wtd_status wtd_set_occ(wtd_ctx *ctx, const double *c_occ);

/* Keep the pair potentials tau_vv' = v_c * (phi_v phi_v') (Eq. trunc) from one
 * apply to the next.  They depend on the occupied orbitals only, so every apply
 * of a Davidson run (Sec. 4) can reuse them; wtd_set_occ and the orbital
 * gradient of wtd_apply_liouville_bwd invalidate them, and the next apply
 * recomputes them.  Off by default (every apply recomputes the pairs).
 * on: 1 keep, 0 recompute every apply.  Host-side flag, ordered with the
 * context stream like every other call.
 * Errors: WTD_ERR_ARG (null), WTD_ERR_SHAPE (on = 1 where the exchange runs
 * row-blocked: Nocc > 128 or a forced row block, whose pair potentials are
 * formed one block pair at a time and do not fit at once).                      */
wtd_status wtd_cache_pairs(wtd_ctx *ctx, int32_t on);

/* Autotuner for the launch shape of the apply (Sec. 4's FFT batching):
 * times whole applies of an nb-trial block for every candidate and keeps the
 * fastest by median of reps timed applies, first the number of workgroups the
 * density reduction of each trial is split over (8, 4, 2, 1), then the number
 * of packed pairs per Poisson batch (the batch allocated at creation, 512 or
 * fewer, and its halvings down to 16, in whole groups of 4 packs).
 * Synchronous; allocates and frees two blocks of nb trial vectors.  The pair
 * potentials do not depend on the batch; the density split changes the
 * summation order of the density response (rounding only).
 * chunk, groups: the chosen values (either may be NULL).
 * Errors: WTD_ERR_ARG (null context, reps outside [1, 100]), WTD_ERR_SHAPE
 * (nb outside [1, max_nb]), WTD_ERR_OOM.                                        */
wtd_status wtd_autotune(wtd_ctx *ctx, int32_t nb, int32_t reps, int32_t *chunk, int32_t *groups);

/* la = P L P a for a block of nb trial sets (Eq. TDDFT_VEXX_TDA's left-hand
 * side, the paper's Sec. 2.1 terms selected by term_mask).
 * a, la: device [nb][nocc][npw][2] in the context precision (double or float);
 * they must not alias.  Asynchronous on the context stream.
 * Errors: WTD_ERR_ARG (null), WTD_ERR_SHAPE (nb < 1 or nb > max_nb).           */
wtd_status wtd_apply_liouville(wtd_ctx *ctx, int32_t nb, const void *a, void *la);

/* The same operator in transition coordinates, always FP64 at the boundary:
 * T = Phi_c^T L Phi_c X, X and T device [nb][nocc][ncond] FP64.  This is the
 * form the Davidson solver applies (Sec. 4).  Asynchronous.                     */
wtd_status wtd_apply_transition(wtd_ctx *ctx, int32_t nb, const double *X, double *T);

/* la = P (D + K1e - K1d + K2e - K2d) P a, the operator of the Z-vector
 * equation (Eq. z-v-eq; the blocks of Eq. TDDFT_VEE summed), with the terms the
 * context's term_mask selects (K2e needs WTD_TERM_K2E, K2d WTD_TERM_K2D; a
 * context created with WTD_TERM_ALL applies the TDA operator here too).
 * K2e: Eq. k2eterm, whose density sum_v' conj(a_v') phi_v' equals K1e's for
 * the real Gamma-point fields.  K2d: Eq. k2dterm, the Poisson-solved products
 * conj(a_v') phi_v of every (v', v), N_b N_occ^2 of them (about 32 times the
 * pair work of K1d at N_b = 16), formed in the pair-potential buffer, so the
 * pair cache of wtd_cache_pairs is dropped by every apply with K2d.
 * Layout, ownership and errors as wtd_apply_liouville.  Asynchronous.           */
wtd_status wtd_apply_full(wtd_ctx *ctx, int32_t nb, const void *a, void *la);

/* Conjugate-gradient solve of the Z-vector equation (Eq. z-v-eq) with the
 * inexact Krylov scheme of Sec. 3.3: each CG system applies the full operator
 * (as wtd_apply_full) until its residual norm falls below lambda_thr and drops
 * K2d from then on (lambda_thr = 0: never).  The nrhs right-hand sides are
 * independent CG systems solved side by side; per iteration the systems still
 * on the full operator form one block apply and those past their switch
 * another.  CG runs in FP64 in transition coordinates (U projected on the
 * conduction orbitals, Z = Phi_c X), the applies in the context precision.
 * Synchronous.  U, Z: device [nrhs][nocc][npw][2] FP64, not aliased; tol:
 * residual 2-norm per system (transition coordinates); resid host [nrhs] (may
 * be NULL); n_iter: iterations of the slowest system; n_exact: iterations in
 * which some system applied the full operator, i.e. the largest count of
 * full-operator iterations of one system (may be NULL).
 * Returns WTD_NOT_CONVERGED (a warning, outputs valid) after max_iter.
 * Errors: WTD_ERR_ARG, WTD_ERR_SHAPE (nrhs outside [1, max_nb]),
 * WTD_ERR_NONFINITE (CG breakdown: the operator is not positive definite).    */
wtd_status wtd_solve_zvector(wtd_ctx *ctx, int32_t nrhs, const double *U, double tol,
                             int32_t max_iter, double lambda_thr, double *Z, double *resid,
                             int32_t *n_iter, int32_t *n_exact);

/* Gradients of E = sum Re(conj(g_la) la), la = L a, with respect to the
 * (re, im) parts of a and of the occupied coefficients c_occ (the derivative of
 * the excitation energy with respect to the orbitals that the Z-vector equation
 * of the paper's Sec. 2.2, Eq. z-v-eq, is built from):
 *   g_a   = W L (W^-1 g_la)  (W: half-sphere weights 1 at m = 0, 2 elsewhere)
 *   g_occ = (2 - delta_m0) x coefficients of gamma_w(r), the derivative with
 *           respect to phi_w(r) of the response and exchange terms; the
 *           orbital-times-trial pair densities it needs are recomputed.
 * a, g_la: device [nb][nocc][npw][2]; g_a: same or NULL; g_occ: device
 * [nocc][npw][2] or NULL; all in the context precision; outputs are
 * overwritten and must not alias the inputs.  nb <= min(max_nb, 16).
 * Asynchronous.  Errors: WTD_ERR_ARG, WTD_ERR_SHAPE.                        */
wtd_status wtd_apply_liouville_bwd(wtd_ctx *ctx, int32_t nb, const void *a, const void *g_la,
                                   void *g_a, void *g_occ);

/* Block Davidson for the nroots lowest eigenpairs of L (Sec. 4; normalisation
 * sum_v <x_v|x_v> = 1 of Eq. ltda).  Synchronous.  Where the exchange is not
 * row-blocked the pair potentials are formed once per call and reused by every
 * apply of the run (as with wtd_cache_pairs).  Each iteration is one device-side
 * step (corrections, their orthonormalisation, the block apply, the subspace
 * matrix and its eigenpairs, Ritz vectors and residuals) followed by one read of
 * the Ritz values and residual norms; on a non-null stream every step after the
 * first is replayed from a HIP graph captured once per (basis size, block size).
 * nb: block size (nroots <= nb <= max_nb); tol: residual 2-norm per root;
 * max_sub: basis cap before restart (<= 0: 4*nb); guess: device
 * [nb][nocc][npw][2] FP64 or NULL (lowest unit transitions).
 * Outputs: omega, resid host [nroots] ascending; x device [nroots][nocc][npw][2]
 * FP64 (may be NULL); n_iter host (may be NULL).
 * Returns WTD_NOT_CONVERGED (a warning) if max_iter is reached.                  */
wtd_status wtd_davidson(wtd_ctx *ctx, int32_t nroots, int32_t nb, double tol, int32_t max_iter,
                        int32_t max_sub, const double *guess, double *omega, double *x,
                        double *resid, int32_t *n_iter);

/* Size of the static device array wtd_davidson_noalloc works in.             */
#define WTD_DAVIDSON_SCRATCH_BYTES ((size_t)64 << 20)

/* wtd_davidson for callers that cannot allocate device memory (code around
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same block Davidson with the same arguments, outputs, warnings and errors,
 * but every buffer of the run (basis and its products, subspace matrix and
 * eigenvectors, Ritz vectors, residuals, corrections, the projected guess and
 * the FP64 copy of the conduction orbitals an FP32 context needs) is carved
 * from one static device array of WTD_DAVIDSON_SCRATCH_BYTES that every GPU
 * the library runs on holds until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine and instantiates no HIP graph (every
 * apply runs eagerly on the workspace wtd_create allocated).  Nothing in the
 * array has to start at zero.  Every call on one GPU uses that GPU's single
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (from other threads or on other contexts) race, and the caller must
 * serialise them.  A run needs about 8 [(2 max_sub + 5 nb) nocc ncond
 * + 21 max_sub^2 + 2 ncond npw] bytes (37 MB at nocc = ncond = 128, nb = 16,
 * max_sub = 64, FP32 bulk, no guess).
 * Errors: as wtd_davidson, plus WTD_ERR_SHAPE naming the bytes needed when the
 * run does not fit in the array.                                               */
wtd_status wtd_davidson_noalloc(wtd_ctx *ctx, int32_t nroots, int32_t nb, double tol,
                                int32_t max_iter, int32_t max_sub, const double *guess,
                                double *omega, double *x, double *resid, int32_t *n_iter);

/* Per-stage timing with HIP events on the context stream (for profiling).
 * wtd_profile_enable(ctx, 1) starts recording; wtd_profile_read copies the
 * accumulated milliseconds and call counts of up to n stages and their names
 * (static strings) and resets them.  Returns the number of stages in *count.  */
wtd_status wtd_profile_enable(wtd_ctx *ctx, int32_t on);
wtd_status wtd_profile_read(wtd_ctx *ctx, int32_t n, double *ms, int64_t *calls,
                            const char **names, int32_t *count);

/* Device bytes held by the context (orbital fields, tables and workspace).      */
wtd_status wtd_workspace_bytes(const wtd_ctx *ctx, size_t *bytes);

/* Process-wide cap on the device memory one context may hold (its workspace,
 * tables and the buffers a first backward call or Davidson adds): a context
 * created afterwards whose allocations would pass `bytes` fails with
 * WTD_ERR_OOM before allocating past it, and so does a later call that would
 * grow it past the cap.  0 (the default) removes the cap.  Contexts that
 * already exist keep their memory.  Thread-safe.                                 */
wtd_status wtd_set_workspace_limit(size_t bytes);

/* Optional input/output checks of one context.  WTD_CHECK_FINITE: every
 * apply (wtd_apply_liouville, wtd_apply_full, wtd_apply_transition,
 * wtd_apply_liouville_bwd) and wtd_set_occ scan their device inputs, and the
 * applies their outputs, for NaN and infinity and return WTD_ERR_NONFINITE
 * naming the array.  The scans synchronise with the context stream, so a
 * context with checks on cannot be captured in a HIP graph.  flags = 0 turns
 * them off (the default).  wtd_create always checks the system arrays
 * (eps_occ, eps_cond, c_occ, c_cond, fxc) and returns WTD_ERR_NONFINITE.
 * Errors: WTD_ERR_ARG (null context, unknown flag).                              */
enum { WTD_CHECK_FINITE = 1 };
wtd_status wtd_set_checks(wtd_ctx *ctx, uint32_t flags);

const char *wtd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WTD_H */
