"""Independent reference routes used to pin the oracle (test code only).

Nothing here calls the oracle or the HIP library.  Each function reaches a
quantity the oracle computes by a different route:

* direct_real_space / direct_coefficients: non-separable direct Fourier sums
  (no FFT) of the plane-wave expansion and its inverse;
* realspace_poisson: the periodic Coulomb potential as an explicit real-space
  convolution with the lattice-summed kernel W(r), O(N_r^2);
* casida_matrix: the TDA matrix in the transition basis assembled without any
  FFT, from pair densities obtained by direct convolution of coefficient lists
  and Coulomb integrals Omega sum_G 4 pi/|G|^2 conj(rho_ab(G)) rho_cd(G).
"""
from __future__ import annotations

import math

import numpy as np


def _gv(mill, cell):
    return np.asarray(mill, dtype=np.float64) * (2.0 * math.pi / np.asarray(cell))[None, :]


def grid_points(cell, n):
    axes = [np.arange(n[i]) * (cell[i] / n[i]) for i in range(3)]
    x, y, z = np.meshgrid(*axes, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def direct_real_space(c_half, mill, cell, n):
    """phi(r) = Omega^-1/2 [c(0) + 2 sum_{m in S+, m != 0} Re(c(m) e^{iG.r})], direct sum."""
    omega = float(np.prod(cell))
    pts = grid_points(cell, n)
    g = _gv(mill, cell)
    ph = np.exp(1j * (pts @ g.T))                     # [N_r][npw]
    c = np.atleast_2d(c_half)
    val = c[:, :1].real.T + 2.0 * np.real(ph[:, 1:] @ c[:, 1:].T)
    out = (val.T / math.sqrt(omega)).reshape((c.shape[0],) + tuple(n))
    return out if np.ndim(c_half) > 1 else out[0]


def direct_coefficients(field, mill, cell):
    """c_F(m) = Omega^1/2 N_r^-1 sum_j F(r_j) e^{-iG_m.r_j}, direct sum."""
    n = field.shape[-3:]
    omega = float(np.prod(cell))
    pts = grid_points(cell, n)
    g = _gv(mill, cell)
    ph = np.exp(-1j * (pts @ g.T))
    f = field.reshape(-1, int(np.prod(n)))
    return (f @ ph) * (math.sqrt(omega) / f.shape[1])


def _box_freq(n):
    return [np.where(np.arange(k) < k / 2, np.arange(k), np.arange(k) - k) for k in n]


def realspace_poisson(rho, cell, n, v_g0=0.0):
    """tau(r_i) = (Omega/N_r) sum_j W(r_i - r_j) rho(r_j) with
    W(r) = Omega^-1 [ sum_{box m != 0} 4 pi/|G_m|^2 cos(G_m.r) + v_g0 ]."""
    omega = float(np.prod(cell))
    nr = int(np.prod(n))
    pts = grid_points(cell, n)
    fr = _box_freq(n)
    mm = np.stack(np.meshgrid(*fr, indexing="ij"), axis=-1).reshape(-1, 3)
    g = _gv(mm, cell)
    g2 = np.sum(g * g, axis=1)
    nz = g2 > 0
    # W at all grid differences: differences of grid points are grid points (periodic)
    w = (np.cos(pts @ g[nz].T) @ (4.0 * math.pi / g2[nz]) + v_g0) / omega   # [N_r]
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3)
    dif = (idx[:, None, :] - idx[None, :, :]) % np.asarray(n)
    flat = (dif[..., 0] * n[1] + dif[..., 1]) * n[2] + dif[..., 2]
    Wm = w[flat]                                                     # [N_r][N_r]
    return ((omega / nr) * (Wm @ rho.reshape(-1))).reshape(n)


def _full_sphere(c_half, mill):
    m = np.asarray(mill)
    c = np.array(c_half, dtype=np.complex128)
    c[0] = c[0].real
    return np.concatenate([m, -m[1:]]), np.concatenate([c, np.conj(c[1:])])


def pair_density_g(ca, cb, mill, omega):
    """Fourier coefficients rho_ab(G) of phi_a phi_b by direct convolution."""
    ma, fa = _full_sphere(ca, mill)
    _, fb = _full_sphere(cb, mill)
    mmax = int(np.abs(ma).max())
    span = 4 * mmax + 1
    s = ma[:, None, :] + ma[None, :, :] + 2 * mmax              # [n][n][3] >= 0
    key = ((s[..., 0] * span) + s[..., 1]) * span + s[..., 2]
    prod = (fa[:, None] * fb[None, :]).ravel() / omega
    k = key.ravel()
    re = np.bincount(k, weights=prod.real, minlength=span ** 3)
    im = np.bincount(k, weights=prod.imag, minlength=span ** 3)
    box = (re + 1j * im).reshape(span, span, span)
    return box, mmax


def coulomb_integral(rab, rcd, mmax, cell, omega, v_g0=0.0):
    """(ab|cd) = Omega sum_G 4 pi/|G|^2 conj(rho_ab(G)) rho_cd(G) (+ v_g0 at G = 0)."""
    span = 4 * mmax + 1
    r = np.arange(span) - 2 * mmax
    b = 2.0 * math.pi / np.asarray(cell)
    g2 = ((r[:, None, None] * b[0]) ** 2 + (r[None, :, None] * b[1]) ** 2
          + (r[None, None, :] * b[2]) ** 2)
    k = np.zeros_like(g2)
    k[g2 > 0] = 4.0 * math.pi / g2[g2 > 0]
    k[2 * mmax, 2 * mmax, 2 * mmax] = v_g0
    return omega * float(np.real(np.sum(np.conj(rab) * rcd * k)))


def casida_matrix(s, with_fxc=True):
    """TDA matrix A[(v,c),(v',c')] = d (eps_c - eps_v) + c_K[(cv|c'v') + (cv|f_xc|c'v')]
    - alpha (cc'|vv'), with the f_xc part as a grid quadrature from direct sums."""
    cell = np.asarray(s.cell, dtype=np.float64)
    omega = float(np.prod(cell))
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    rcv = {}
    for v in range(nocc):
        for c in range(nc):
            rcv[v, c], mmax = pair_density_g(s.c_cond[c], s.c_occ[v], s.mill, omega)
    rcc = {}
    for c in range(nc):
        for c2 in range(c, nc):
            rcc[c, c2], _ = pair_density_g(s.c_cond[c], s.c_cond[c2], s.mill, omega)
            rcc[c2, c] = rcc[c, c2]
    rvv = {}
    for v in range(nocc):
        for v2 in range(v, nocc):
            rvv[v, v2], _ = pair_density_g(s.c_occ[v], s.c_occ[v2], s.mill, omega)
            rvv[v2, v] = rvv[v, v2]
    fx = None
    if with_fxc:
        po = direct_real_space(s.c_occ, s.mill, cell, s.n).reshape(nocc, -1)
        pc = direct_real_space(s.c_cond, s.mill, cell, s.n).reshape(nc, -1)
        prod = (pc[None, :, :] * po[:, None, :]).reshape(nocc * nc, -1)
        nr = prod.shape[1]
        fx = (omega / nr) * (prod * s.fxc.reshape(1, -1)) @ prod.T
    dim = nocc * nc
    A = np.zeros((dim, dim))
    for i in range(dim):
        v, c = divmod(i, nc)
        for j in range(dim):
            v2, c2 = divmod(j, nc)
            val = 0.0
            if i == j:
                val += s.eps_cond[c] - s.eps_occ[v]
            if s.c_k != 0.0:
                val += s.c_k * coulomb_integral(rcv[v, c], rcv[v2, c2], mmax, cell, omega,
                                                s.v_g0)
                if fx is not None:
                    val += s.c_k * fx[i, j]
            if s.alpha != 0.0:
                val -= s.alpha * coulomb_integral(rcc[c, c2], rvv[v, v2], mmax, cell,
                                                  omega, s.v_g0)
            A[i, j] = val
    return A


def casida_b_matrix(s, with_fxc=True):
    """Off-diagonal block of Eq. TDDFT_VEE for real (Gamma-point) orbitals:
    B[(v,c),(v',c')] = c_K[(cv|v'c') + (cv|f_xc|v'c')] - alpha (cv'|c'v), the
    matrix of K2e - K2d in the transition basis, from direct sums."""
    cell = np.asarray(s.cell, dtype=np.float64)
    omega = float(np.prod(cell))
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    rcv = {}
    for v in range(nocc):
        for c in range(nc):
            rcv[v, c], mmax = pair_density_g(s.c_cond[c], s.c_occ[v], s.mill, omega)
    fx = None
    if with_fxc:
        po = direct_real_space(s.c_occ, s.mill, cell, s.n).reshape(nocc, -1)
        pc = direct_real_space(s.c_cond, s.mill, cell, s.n).reshape(nc, -1)
        prod = (pc[None, :, :] * po[:, None, :]).reshape(nocc * nc, -1)
        nr = prod.shape[1]
        fx = (omega / nr) * (prod * s.fxc.reshape(1, -1)) @ prod.T
    dim = nocc * nc
    B = np.zeros((dim, dim))
    for i in range(dim):
        v, c = divmod(i, nc)
        for j in range(dim):
            v2, c2 = divmod(j, nc)
            val = 0.0
            if s.c_k != 0.0:
                # (cv|v'c'): pair densities phi_c phi_v and phi_v' phi_c' (real orbitals)
                val += s.c_k * coulomb_integral(rcv[v, c], rcv[v2, c2], mmax, cell, omega,
                                                s.v_g0)
                if fx is not None:
                    val += s.c_k * fx[i, j]
            if s.alpha != 0.0:
                # (cv'|c'v): pair densities phi_c phi_v' and phi_c' phi_v
                val -= s.alpha * coulomb_integral(rcv[v2, c], rcv[v, c2], mmax, cell, omega,
                                                  s.v_g0)
            B[i, j] = val
    return B
