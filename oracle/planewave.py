"""Plane-wave conventions at the Gamma point (oracle).

Conventions (Hartree atomic units, Coulomb kernel 1/|r - r'|):

* Cell volume Omega = L0 L1 L2, grid r_j = (L0 i0/n0, L1 i1/n1, L2 i2/n2),
  N_r = n0 n1 n2, G_m = 2 pi (m0/L0, m1/L1, m2/L2).
* A real orbital is phi(r) = Omega^(-1/2) sum_{m in S} c(m) e^{i G_m . r} with
  c(-m) = conj(c(m)); only the half sphere S+ is stored (m = 0 first).
* Gamma inner product <f|g> = sum_{m in S+} w_m Re(conj(f_m) g_m), w_0 = 1,
  w_m = 2 otherwise; it equals (Omega/N_r) sum_j f(r_j) g(r_j).
* Forward coefficients of a real field F on the grid:
  c_F(m) = Omega^(1/2) (1/N_r) sum_j F(r_j) e^{-i G_m . r_j}.
* Poisson: (v_c * rho)(r_j) = sum_{m != 0} 4 pi/|G_m|^2 rho^(m) e^{i G_m r_j}
  + v_g0 rho^(0), with rho^ the normalised forward transform and the sum over
  the whole FFT box (box index k maps to m = k for k < n/2, k - n otherwise).

The Gamma-point restriction and real orbitals are those of Sec. 2 of the paper.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

_WORKERS = -1


def gvectors(mill, cell):
    """Cartesian G vectors [npw][3] for Miller indices and an orthorhombic cell."""
    b = 2.0 * math.pi / np.asarray(cell, dtype=np.float64)
    return np.asarray(mill, dtype=np.float64) * b[None, :]


def gamma_inner(f, g):
    """<f|g> over the last axis of half-sphere coefficient arrays."""
    npw = f.shape[-1]
    w = np.full(npw, 2.0)
    w[0] = 1.0
    return np.sum(w * (f.real * g.real + f.imag * g.imag), axis=-1)


def gamma_overlap(f, g):
    """<f_i|g_j> for every pair of half-sphere coefficient rows f [nf][npw] and
    g [ng][npw], as one weighted matrix product (result [nf][ng])."""
    f = np.asarray(f, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    w = np.full(f.shape[-1], 2.0)
    w[0] = 1.0
    return (f.real * w) @ g.real.T + (f.imag * w) @ g.imag.T


def _box(c_half, mill, n):
    """Place half-sphere coefficients and their conjugates in the FFT box."""
    lead = c_half.shape[:-1]
    box = np.zeros(lead + tuple(n), dtype=np.complex128)
    m = np.asarray(mill)
    kp = tuple(np.mod(m[:, i], n[i]) for i in range(3))
    km = tuple(np.mod(-m[:, i], n[i]) for i in range(3))
    c = c_half.copy()
    c[..., 0] = c[..., 0].real          # the G = 0 coefficient of a real function is real
    box[(Ellipsis,) + km] = np.conj(c)
    box[(Ellipsis,) + kp] = c           # m = 0 written last (its own mirror)
    return box


def real_space(c_half, mill, cell, n, chunk=16):
    """phi(r_j) on the grid for every leading index of c_half ([..., npw])."""
    omega = float(np.prod(cell))
    nr = int(np.prod(n))
    c_half = np.asarray(c_half, dtype=np.complex128)
    lead = c_half.shape[:-1]
    flat = c_half.reshape(-1, c_half.shape[-1])
    out = np.empty((flat.shape[0],) + tuple(n))
    for i in range(0, flat.shape[0], chunk):
        box = _box(flat[i:i + chunk], mill, n)
        f = sfft.ifftn(box, axes=(-3, -2, -1), workers=_WORKERS)
        out[i:i + chunk] = f.real * (nr / math.sqrt(omega))
    return out.reshape(lead + tuple(n))


def coefficients(field, mill, cell):
    """Half-sphere coefficients c_F(m) of real fields [..., n0, n1, n2]."""
    field = np.asarray(field, dtype=np.float64)
    n = field.shape[-3:]
    lead = field.shape[:-3]
    omega = float(np.prod(cell))
    nr = int(np.prod(n))
    m = np.asarray(mill)
    k = tuple(np.mod(m[:, i], n[i]) for i in range(3))
    flat = field.reshape((-1,) + tuple(n))
    out = np.empty((flat.shape[0], m.shape[0]), dtype=np.complex128)
    for i in range(flat.shape[0]):
        ft = sfft.fftn(flat[i], workers=_WORKERS)
        out[i] = ft[k] * (math.sqrt(omega) / nr)
    return out.reshape(lead + (m.shape[0],))


def coulomb_kernel(cell, n, v_g0=0.0):
    """4 pi / |G|^2 on the whole box (real-FFT half layout), v_g0 at G = 0."""
    b = 2.0 * math.pi / np.asarray(cell, dtype=np.float64)
    f0 = sfft.fftfreq(n[0], 1.0 / n[0]) * b[0]
    f1 = sfft.fftfreq(n[1], 1.0 / n[1]) * b[1]
    f2 = np.arange(n[2] // 2 + 1) * b[2]
    g2 = f0[:, None, None] ** 2 + f1[None, :, None] ** 2 + f2[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        k = 4.0 * math.pi / g2
    k[0, 0, 0] = v_g0
    return k


def poisson(rho, kernel):
    """v_c * rho on the grid for real fields rho [..., n0, n1, n2]."""
    n = rho.shape[-3:]
    rk = sfft.rfftn(rho, axes=(-3, -2, -1), workers=_WORKERS)
    return sfft.irfftn(rk * kernel, s=n, axes=(-3, -2, -1), workers=_WORKERS)
