"""Conjugate-gradient solve of the Z-vector equation (oracle).

The paper obtains the Z-vectors of the excited-state forces from
(D + K1e - K1d + K2e - K2d) Z = U (Eq. z-v-eq) by conjugate gradients, and
accelerates it with an inexact Krylov scheme (Sec. 3.3): the exact operator is
applied until the residual vector falls below a threshold lambda_thr, and from
then on an approximate operator without the K2d term.

Readings taken here (the paper gives no further detail):

* The solve runs in transition coordinates X [nocc][nc] (Z_v = sum_c X_vc phi_c,
  the right-hand side projected the same way), where the operator is a
  symmetric matrix and the Gamma inner product is the Euclidean one.
* Plain (Hestenes-Stiefel) CG from Z = 0 for each right-hand side on its own;
  "residual" is the recurrence residual r_k, its size the 2-norm.
* The switch to the approximate operator happens once, at the first iteration
  whose residual norm is below lambda_thr (lambda_thr = 0: never); iterations
  stop when the norm is at or below tol, or after max_iter.
"""
from __future__ import annotations

import numpy as np

from .liouville import TERM_FULL, TERM_K2D, apply_transition


def cg_inexact(matvec_exact, matvec_approx, rhs, tol=1e-8, max_iter=200, lambda_thr=0.0):
    """Solve A z = rhs for one vector; returns (z, residual norm, iterations, exact applies)."""
    b = np.asarray(rhs, dtype=np.float64).ravel()
    z = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    use_exact = True
    n_exact = 0
    it = 0
    while np.sqrt(rr) > tol and it < max_iter:
        if use_exact and lambda_thr > 0.0 and np.sqrt(rr) < lambda_thr:
            use_exact = False
        if use_exact:
            ap = matvec_exact(p)
            n_exact += 1
        else:
            ap = matvec_approx(p)
        step = rr / float(p @ ap)
        z = z + step * p
        r = r - step * ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return z, float(np.sqrt(rr)), it, n_exact


def solve_zvector_transition(s, U, tol=1e-8, max_iter=200, lambda_thr=0.0):
    """Z-vectors for right-hand sides U [nrhs][nocc][nc] in transition coordinates.

    The right-hand sides are solved side by side, one CG each, with one shared
    operator per iteration: the approximate operator is taken from the first
    iteration at which every unconverged residual norm is below lambda_thr (for
    one right-hand side this is the rule of cg_inexact).  A converged system is
    left as it is.  Returns (Z [nrhs][nocc][nc], residual norms, iterations,
    applies of the exact operator)."""
    U = np.asarray(U, dtype=np.float64)
    nrhs, nocc, nc = U.shape
    Z = np.zeros((nrhs, nocc * nc))
    R = U.reshape(nrhs, -1).copy()
    P = R.copy()
    rr = np.sum(R * R, axis=1)
    active = np.sqrt(rr) > tol
    use_exact = True
    n_exact = 0
    it = 0
    while active.any() and it < max_iter:
        if use_exact and lambda_thr > 0.0 and np.all(np.sqrt(rr[active]) < lambda_thr):
            use_exact = False
        terms = TERM_FULL if use_exact else TERM_FULL & ~TERM_K2D
        AP = apply_transition(s, P.reshape(nrhs, nocc, nc), terms=terms).reshape(nrhs, -1)
        n_exact += int(use_exact)
        for k in np.flatnonzero(active):
            step = rr[k] / float(P[k] @ AP[k])
            Z[k] += step * P[k]
            R[k] -= step * AP[k]
            rr_new = float(R[k] @ R[k])
            P[k] = R[k] + (rr_new / rr[k]) * P[k]
            rr[k] = rr_new
        active = np.sqrt(rr) > tol
        it += 1
    return Z.reshape(nrhs, nocc, nc), np.sqrt(rr), it, n_exact
