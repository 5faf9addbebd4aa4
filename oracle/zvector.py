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

    Each right-hand side is its own CG solve (cg_inexact) with its own switch
    to the approximate operator (Sec. 3.3 states the switch for one CG).
    Returns (Z [nrhs][nocc][nc], residual norms, iterations, exact applies),
    the last two as the maxima over the right-hand sides."""
    U = np.asarray(U, dtype=np.float64)
    nrhs, nocc, nc = U.shape

    def op(terms):
        def mv(x):
            return apply_transition(s, x.reshape(1, nocc, nc), terms=terms).ravel()
        return mv

    exact = op(TERM_FULL)
    approx = op(TERM_FULL & ~TERM_K2D)
    Z = np.zeros((nrhs, nocc * nc))
    rn = np.zeros(nrhs)
    its, nex = [], []
    for k in range(nrhs):
        Z[k], rn[k], it, ne = cg_inexact(exact, approx, U[k], tol=tol, max_iter=max_iter,
                                         lambda_thr=lambda_thr)
        its.append(it)
        nex.append(ne)
    return Z.reshape(nrhs, nocc, nc), rn, max(its), max(nex)
