"""Adjoint of the Liouville apply (oracle): gradients of E = Re sum conj(g) (L a).

This is the building block of the orbital derivative u_v of the paper's
Eq. z-v-eq and SI Eq. Zvectoreq (the derivative of A^T (D + K1e - K1d) A with
respect to the occupied orbitals); here it is written for a general cotangent g.

Gradients are returned as complex arrays whose real and imaginary parts are
dE/dRe and dE/dIm of the half-sphere coefficients.

* With respect to a: L is linear and symmetric in the Gamma inner product
  <x|y> = x^T W y (W the half-sphere weights 1 and 2), so
  dE/da = L^T g = W L (W^-1 g).
* With respect to the occupied coefficients, through the real-space fields
  phi_w(r_j) (D and the projector do not depend on them):
    g~_bv  = real-space field of sum_c (phi_c . g_bv) phi_c   (Euclidean dot)
    drho_b = sum_v phi_v a~_bv,  drho^g_b = sum_v phi_v g~_bv,  F = v_c * + f_xc
    M_vv'  = sum_b g~_bv a~_bv'
    gamma_w = c_K sum_b [ g~_bw F(drho_b) + a~_bw F(drho^g_b) ]
              - alpha sum_v' phi_v' v_c * (M_wv' + M_v'w)
  and, with dE = (Omega/N_r) sum_j dphi_w(r_j) gamma_w(r_j),
    dE/dc_w(m) = (2 - delta_m0) c_gamma(m),  c_gamma the forward coefficients
  of gamma_w (imaginary part zero at m = 0).
"""
from __future__ import annotations

import numpy as np

from .liouville import TERM_ALL, TERM_K1D, TERM_K1E, apply_liouville
from .planewave import coefficients, coulomb_kernel, gamma_overlap, poisson, real_space


def _weights(npw):
    w = np.full(npw, 2.0)
    w[0] = 1.0
    return w


def grad_a(s, a, g, terms=TERM_ALL):
    """dE/da = W L (W^-1 g) for E = Re sum conj(g) L a (independent of a)."""
    del a
    w = _weights(g.shape[-1])
    out = w * apply_liouville(s, g / w, terms=terms)
    out[..., 0] = out[..., 0].real
    return out


def grad_occ(s, a, g, terms=TERM_ALL, occ=None):
    """dE/dc_occ for E = Re sum conj(g) L a; shape [nocc][npw] complex."""
    a = np.asarray(a, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    cell, n, mill = np.asarray(s.cell, dtype=np.float64), tuple(s.n), s.mill
    c_occ = s.c_occ if occ is None else occ
    c_cond = s.c_cond
    nb, nocc, npw = a.shape
    k1e = bool(terms & TERM_K1E) and s.c_k != 0.0
    k1d = bool(terms & TERM_K1D) and s.alpha != 0.0
    gamma = np.zeros((nocc,) + n)
    if not (k1e or k1d):
        return np.zeros((nocc, npw), dtype=np.complex128)

    S = gamma_overlap(a.reshape(-1, a.shape[-1]), c_cond).reshape(a.shape[0], a.shape[1], -1)
    at = real_space(np.einsum("bvc,cm->bvm", S, c_cond), mill, cell, n)
    G = np.einsum("cm,bvm->bvc", c_cond.real, g.real) + np.einsum("cm,bvm->bvc", c_cond.imag,
                                                                   g.imag)
    gt = real_space(np.einsum("bvc,cm->bvm", G, c_cond), mill, cell, n)
    phi = real_space(c_occ, mill, cell, n)
    kern = coulomb_kernel(cell, n, s.v_g0)

    if k1e:
        drho = np.stack([np.einsum("vxyz,vxyz->xyz", phi, at[b]) for b in range(nb)])
        drho_g = np.stack([np.einsum("vxyz,vxyz->xyz", phi, gt[b]) for b in range(nb)])
        F = poisson(drho, kern) + s.fxc[None] * drho
        Fg = poisson(drho_g, kern) + s.fxc[None] * drho_g
        for w_ in range(nocc):
            gamma[w_] += s.c_k * np.sum(gt[:, w_] * F + at[:, w_] * Fg, axis=0)
    if k1d:
        for w_ in range(nocc):
            for vp in range(nocc):
                m = np.sum(gt[:, w_] * at[:, vp] + gt[:, vp] * at[:, w_], axis=0)
                gamma[w_] -= s.alpha * phi[vp] * poisson(m, kern)

    w = _weights(npw)
    out = w * coefficients(gamma, mill, cell)
    out[:, 0] = out[:, 0].real
    return out


def energy(s, a, g, terms=TERM_ALL, occ=None):
    """E = Re sum conj(g) (L a), the scalar whose gradients the adjoint returns."""
    la = apply_liouville(s, a, terms=terms, occ=occ)
    return float(np.sum(g.real * la.real + g.imag * la.imag))
