"""A posteriori certificates of eigenpairs (test code only).

An eigensolver's vectors are not unique (sign, rotations inside degenerate
roots), so a returned Ritz pair is checked by what it must satisfy rather than
compared entry by entry: the Rayleigh-Ritz values of the operator on the span
of the returned vectors (the excitation energy as a Rayleigh quotient,
Sec. 2.3), the residual norm of each Ritz pair, and two classical bounds on the
distance to the exact eigenvalue:

* Weinstein: some eigenvalue lies within ||r|| of a Rayleigh quotient theta of
  a unit vector with residual r;
* Kato-Temple: if the open interval (a, b) around theta contains exactly one
  eigenvalue lam, then |theta - lam| <= ||r||^2 / min(theta - a, b - theta).
  Here a and b come from the neighbouring Ritz values and their Weinstein
  intervals (the lowest root has no eigenvalue below it; the highest root of
  the set has no known upper neighbour and gets no Kato-Temple bound).

The operator enters as a matvec on an (n, k) block, so the same code runs on a
dense matrix (pinned against eigh) and on the oracle in transition coordinates.
"""
from __future__ import annotations

import numpy as np

import oracle


def rayleigh_ritz(matvec, V):
    """Rayleigh-Ritz of a symmetric operator on span(V), V [n][k] (real).

    Returns (theta [k] ascending, Y [n][k] orthonormal Ritz vectors, rnorm [k]
    residual norms ||A y - theta y||, kt [k] Kato-Temple bounds, None for the
    highest root)."""
    V = np.asarray(V, dtype=np.float64)
    Q, _ = np.linalg.qr(V)
    AQ = np.asarray(matvec(Q), dtype=np.float64)
    H = Q.T @ AQ
    H = 0.5 * (H + H.T)
    theta, U = np.linalg.eigh(H)
    Y = Q @ U
    R = AQ @ U - Y * theta[None, :]
    rn = np.linalg.norm(R, axis=0)
    k = theta.size
    kt = []
    for i in range(k - 1):
        below = theta[i] - (theta[i - 1] + rn[i - 1]) if i > 0 else np.inf
        above = (theta[i + 1] - rn[i + 1]) - theta[i]
        gap = min(below, above)
        kt.append(rn[i] ** 2 / gap if gap > 0 else np.inf)
    kt.append(None)
    return theta, Y, rn, kt


def transition_matvec(s, terms=oracle.TERM_ALL):
    """The oracle's operator in transition coordinates as a matvec on [nocc nc][k]."""
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]

    def mv(V):
        k = V.shape[1]
        out = oracle.apply_transition(s, V.T.reshape(k, nocc, nc), terms=terms)
        return out.reshape(k, nocc * nc).T
    return mv


def transition_coordinates(s, x):
    """Half-sphere coefficient sets x [k][nocc][npw] (complex) -> X [nocc nc][k],
    X_vc = <phi_c|x_v> (the sets lie in the conduction span)."""
    k, nocc, npw = x.shape
    X = oracle.gamma_overlap(x.reshape(k * nocc, npw), s.c_cond)
    return X.reshape(k, -1).T
