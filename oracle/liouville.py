"""The Tamm-Dancoff Liouville operator L = D + K1e - K1d applied to trial sets (oracle),
and the full operator D + K1e - K1d + K2e - K2d of the Z-vector equation.

Follows Sec. 2.1 of the paper: the D term (Eq. dterm), the density-response
term K1e with f_Hxc = v_c + f_xc (Eq. k1eterm), the exact-exchange term K1d
(Eq. k1d) built from occupied-occupied pair potentials
tau_vv'(r) = int v_c(r, r') phi_v'(r') phi_v(r') (the N_occ^2 integrations of
Sec. 3.2, Eq. trunc), the projector P_c (defined after Eq. k2dterm) and the TDA
problem of Eq. TDDFT_VEXX_TDA.

Readings of the paper taken here (the paper is silent or general on these):

* Projector: the "unoccupied manifold" of a synthetic system is the span of the
  supplied conduction orbitals, P = sum_c |phi_c><phi_c|, and H_KS acts
  spectrally, H_KS phi_n = eps_n phi_n, so D = P (H_KS - eps_v) P has entries
  eps_c - eps_v in the transition basis.  With a complete basis this is the
  paper's 1 - sum_v |phi_v><phi_v|; ``projector="complement"`` uses that form.
  The input is projected too (L is applied as P L P), so L is symmetric for any
  input.
* Spin: closed-shell singlet sector of two identical spin channels, so the
  K1e term carries a factor c_K (2.0; 0.0 drops it, as in the spin-flip
  problem with the exchange term only).  f_xc is an input field.
* Exchange pairs: the paper's K1d, occupied-occupied pair densities
  phi_v phi_v', Poisson-solved and multiplied by the trial orbital a_v'.
* Coulomb G = 0: the kernel value there is the parameter v_g0 (0 drops it).
* The operator is defined on the FFT grid: products are formed at grid points
  and integrals are grid quadratures.

* K2e and K2d (Eqs. k2eterm, k2dterm) enter the Z-vector equation (Eq.
  z-v-eq) and the off-diagonal blocks of Eq. TDDFT_VEE.  K2e's density is
  sum_v' conj(a_v') phi_v', K2d's pairs are conj(a_v') phi_v, Poisson-solved
  and multiplied by phi_v'.  At the Gamma point every field here is real, so
  K2e equals K1e; the conjugates are kept to follow the equations.

Steps, for every trial b and occupied v (Hartree units):
 1. S_cv = <phi_c|a_v>, a~_v = sum_c phi_c S_cv
 2. phi_v(r_j), a~_v(r_j) on the grid
 3. drho(r_j) = sum_v phi_v(r_j) a~_v(r_j)
 4. V(r_j) = c_K [ (v_c * drho)(r_j) + f_xc(r_j) drho(r_j) ]
 5. tau_vv'(r_j) = (v_c * (phi_v phi_v'))(r_j)
 6. R_v(r_j) = phi_v(r_j) V(r_j) - alpha sum_v' tau_vv'(r_j) a~_v'(r_j)
    (full operator: V also carries K2e's density, and R_v also gets
    - alpha sum_v' phi_v'(r_j) (v_c * (conj(a~_v') phi_v))(r_j), the K2d term)
 7. la_v = sum_c phi_c [ (eps_c - eps_v) S_cv + (Omega/N_r) sum_j phi_c(r_j) R_v(r_j) ]
"""
from __future__ import annotations

import numpy as np

from .planewave import coefficients, coulomb_kernel, gamma_overlap, poisson, real_space

TERM_D = 1
TERM_K1E = 2
TERM_K1D = 4
TERM_ALL = 7      # the TDA operator D + K1e - K1d
TERM_K2E = 8
TERM_K2D = 16
TERM_FULL = 31    # D + K1e - K1d + K2e - K2d (Eq. z-v-eq)


def apply_liouville(s, a, terms=TERM_ALL, rows=None, projector="span", occ=None, progress=None):
    """la = L a for a trial block a [nb][nocc][npw] (complex half-sphere coefficients).

    ``s`` carries cell, n, mill, c_occ, c_cond, eps_occ, eps_cond, fxc, alpha,
    c_k and v_g0.  ``rows`` restricts the output to a list of occupied indices
    v (the result then has shape [nb][len(rows)][npw]); the sum over v' always
    runs over every occupied orbital.  ``occ`` overrides the occupied
    coefficients (used by the rotation-invariance check).  ``progress``, if
    given, is called with a short message as each step completes.
    """
    say = progress if progress is not None else (lambda msg: None)
    a = np.asarray(a, dtype=np.complex128)
    cell, n, mill = np.asarray(s.cell, dtype=np.float64), tuple(s.n), s.mill
    c_occ = s.c_occ if occ is None else occ
    c_cond = s.c_cond
    nb, nocc, npw = a.shape
    assert c_occ.shape == (nocc, npw)
    rows = list(range(nocc)) if rows is None else [int(v) for v in rows]
    omega = float(np.prod(cell))
    nr = int(np.prod(n))

    # step 1: project the input onto the unoccupied manifold
    if projector == "span":
        S = gamma_overlap(a.reshape(nb * nocc, npw), c_cond).reshape(nb, nocc, -1)  # [nb][nocc][nc]
        a_t = np.einsum("bvc,cm->bvm", S, c_cond)
    elif projector == "complement":
        O = gamma_overlap(a.reshape(nb * nocc, npw), c_occ).reshape(nb, nocc, nocc)
        a_t = a - np.einsum("bvu,um->bvm", O, c_occ)
    else:
        raise ValueError(projector)

    # step 2: real space
    phi = real_space(c_occ, mill, cell, n)                                  # [nocc][n]
    at = real_space(a_t, mill, cell, n)                                     # [nb][nocc][n]
    say("oracle: orbitals and projected trials on the grid")

    # steps 3-4: density response and its Hartree + f_xc potential
    V = None
    if terms & (TERM_K1E | TERM_K2E) and s.c_k != 0.0:
        kern = coulomb_kernel(cell, n, s.v_g0)
        drho = np.zeros((nb,) + n)
        if terms & TERM_K1E:       # sum_v' conj(phi_v') a_v'
            drho += np.stack([np.einsum("vxyz,vxyz->xyz", np.conj(phi), at[b]) for b in range(nb)])
        if terms & TERM_K2E:       # sum_v' conj(a_v') phi_v'
            drho += np.stack([np.einsum("vxyz,vxyz->xyz", np.conj(at[b]), phi) for b in range(nb)])
        V = s.c_k * (poisson(drho, kern) + s.fxc[None] * drho)
        say("oracle: density response potential")

    # steps 5-6: R_v(r) for the requested rows
    R = np.zeros((nb, len(rows)) + n)
    if V is not None:
        for i, v in enumerate(rows):
            R[:, i] += phi[v][None] * V
    if terms & TERM_K1D and s.alpha != 0.0:
        kern = coulomb_kernel(cell, n, s.v_g0)
        for i, v in enumerate(rows):
            tau = poisson(phi[v][None] * phi, kern)                         # [nocc][n]
            for b in range(nb):
                R[b, i] -= s.alpha * np.einsum("uxyz,uxyz->xyz", tau, at[b])
            say(f"oracle: exchange for row {v}")
    if terms & TERM_K2D and s.alpha != 0.0:
        kern = coulomb_kernel(cell, n, s.v_g0)
        for i, v in enumerate(rows):
            for b in range(nb):
                w = poisson(np.conj(at[b]) * phi[v][None], kern)          # [v'][n]
                R[b, i] -= s.alpha * np.einsum("uxyz,uxyz->xyz", phi, w)
            say(f"oracle: K2d for row {v}")

    # step 7: back to the projected plane-wave space
    if projector == "span":
        phic = real_space(c_cond, mill, cell, n)                            # [nc][n]
        Q = (omega / nr) * (R.reshape(nb * len(rows), nr) @ phic.reshape(-1, nr).T)
        Q = Q.reshape(nb, len(rows), -1)
        T = Q
        if terms & TERM_D:
            de = s.eps_cond[None, None, :] - np.asarray(s.eps_occ)[rows][None, :, None]
            T = T + de * S[:, rows, :]
        return np.einsum("bvc,cm->bvm", T, c_cond)

    # paper-literal projector 1 - sum_v |phi_v><phi_v| with spectral H_KS over
    # the supplied occupied and conduction orbitals
    out = coefficients(R, mill, cell)                                       # [nb][rows][npw]
    if terms & TERM_D:
        orbs = np.concatenate([c_occ, c_cond])
        eps = np.concatenate([s.eps_occ, s.eps_cond])
        at_r = a_t[:, rows]
        proj = gamma_overlap(at_r.reshape(-1, npw), orbs).reshape(nb, len(rows), -1)
        h_at = np.einsum("bvn,n,nm->bvm", proj, eps, orbs)
        out = out + h_at - np.asarray(s.eps_occ)[rows][None, :, None] * at_r
    O = gamma_overlap(out.reshape(-1, npw), c_occ).reshape(nb, len(rows), nocc)
    return out - np.einsum("bvu,um->bvm", O, c_occ)


def transition_diagonal(s):
    """eps_c - eps_v as an array [nocc][nc] (the D term in the transition basis)."""
    return np.asarray(s.eps_cond)[None, :] - np.asarray(s.eps_occ)[:, None]


def apply_transition(s, X, terms=TERM_ALL):
    """L in transition coordinates: X [nb][nocc][nc] -> Phi_c^T L (Phi_c X).

    Exactly equivalent to apply_liouville on a_v = sum_c X_vc phi_c because the
    conduction orbitals are orthonormal."""
    X = np.asarray(X, dtype=np.float64)
    a = np.einsum("bvc,cm->bvm", X, s.c_cond)
    la = apply_liouville(s, a, terms=terms)
    nb, nocc, npw = la.shape
    return gamma_overlap(la.reshape(nb * nocc, npw), s.c_cond).reshape(nb, nocc, -1)
