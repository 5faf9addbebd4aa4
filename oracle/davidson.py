"""Block Davidson eigensolver for the lowest roots of L (oracle).

The paper diagonalises the Liouville super-operator iteratively with the
Davidson method (Sec. 4) under the normalisation sum_v <a_v|a_v> = 1
(Eq. ltda).  It gives no further detail, so this is the standard block variant
with a diagonal preconditioner:

* guess: the nb unit transitions with the lowest eps_c - eps_v (ties: smaller
  c, then larger v), or a supplied block, orthonormalised;
* each iteration: W = L V for the new vectors; H = V^T W symmetrised; eigh;
  Ritz vectors x_k = V y_k and residuals r_k = W y_k - theta_k x_k for the nb
  lowest pairs; stop when ||r_k|| <= tol for the nroots lowest;
* corrections t_k = r_k / (d - theta_k) for the unconverged k < nb, where d is
  the transition diagonal and each denominator's magnitude is floored at 1e-3
  with its sign kept (zero counts as positive);
* classical Gram-Schmidt, applied twice, against V and the earlier accepted
  corrections; a correction whose norm falls below 1e-10 is dropped;
* when the basis would exceed max_sub vectors it is collapsed to the nb
  lowest Ritz vectors (with W collapsed alongside);
* when every correction is dropped (the basis already holds them) the run
  stops unconverged and reports the iteration it stopped at.
"""
from __future__ import annotations

import numpy as np

from .liouville import TERM_ALL, apply_transition, transition_diagonal


def _guess(diag, nb):
    nocc, nc = diag.shape
    v, c = np.meshgrid(np.arange(nocc), np.arange(nc), indexing="ij")
    order = np.lexsort(((-v).ravel(), c.ravel(), diag.ravel()))
    V = np.zeros((diag.size, nb))
    V[order[:nb], np.arange(nb)] = 1.0
    return V


def davidson(matvec, diag, nroots, nb, tol=1e-8, max_iter=100, max_sub=None, guess=None):
    """Lowest ``nroots`` eigenpairs of the symmetric operator ``matvec``.

    matvec maps an (n, k) block to (n, k); diag is the preconditioner diagonal
    (any shape of size n).  Returns (theta[nroots], X[n][nroots], rnorm[nroots],
    n_iter, converged)."""
    d = np.asarray(diag, dtype=np.float64).ravel()
    n = d.size
    nb = min(nb, n)
    max_sub = max(max_sub or 4 * nb, 2 * nb)
    max_sub = min(max_sub, n)
    if guess is None:
        V = _guess(np.asarray(diag).reshape(-1, 1) if np.ndim(diag) == 1 else diag, nb)
    else:
        V = np.array(guess, dtype=np.float64).reshape(n, -1)
        for _ in range(2):
            V, _ = np.linalg.qr(V)
    W = matvec(V)
    theta = rn = X = None
    it = 0
    for it in range(1, max_iter + 1):
        H = V.T @ W
        H = 0.5 * (H + H.T)
        th, Y = np.linalg.eigh(H)
        k = min(nb, V.shape[1])
        Yk = Y[:, :k]
        X = V @ Yk
        R = W @ Yk - X * th[None, :k]
        rn = np.linalg.norm(R, axis=0)
        theta = th[:k]
        if np.all(rn[:nroots] <= tol):
            return theta[:nroots], X[:, :nroots], rn[:nroots], it, True
        T = []
        for j in range(k):
            if rn[j] <= tol:
                continue
            den = d - th[j]
            small = np.abs(den) < 1e-3
            den[small] = np.where(den[small] < 0.0, -1e-3, 1e-3)
            T.append(R[:, j] / den)
        T = np.array(T).T
        if V.shape[1] + T.shape[1] > max_sub:
            V, W = X.copy(), W @ Yk
        accepted = []
        for j in range(T.shape[1]):
            t = T[:, j].copy()
            basis = np.column_stack([V] + accepted) if accepted else V
            for _ in range(2):
                t -= basis @ (basis.T @ t)
            nt = np.linalg.norm(t)
            if nt < 1e-10:
                continue
            accepted.append(t / nt)
        if not accepted:
            # every correction lies in the basis already: nothing left to add
            break
        Tn = np.column_stack(accepted)
        V = np.column_stack([V, Tn])
        W = np.column_stack([W, matvec(Tn)])
    return theta[:nroots], X[:, :nroots], rn[:nroots], it, False


def davidson_transition(s, nroots, nb, tol=1e-8, max_iter=100, max_sub=None,
                        terms=TERM_ALL, guess=None):
    """Davidson on L in transition coordinates X [nocc][nc] (see apply_transition)."""
    diag = transition_diagonal(s)
    nocc, nc = diag.shape

    def matvec(V):
        Xb = V.T.reshape(-1, nocc, nc)
        return apply_transition(s, Xb, terms=terms).reshape(V.shape[1], -1).T

    return davidson(matvec, diag, nroots, nb, tol=tol, max_iter=max_iter,
                    max_sub=max_sub, guess=guess)
