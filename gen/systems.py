"""Seeded synthetic systems and trial blocks.

The paper's ground states (Quantum ESPRESSO runs of point-defect supercells) are
not available, so every workload is synthetic.  The recipe:

* Plane-wave sphere: Miller indices m with |G_m|^2 <= E_cut (Ry, |G| in 1/bohr),
  G_m = 2*pi*(m0/L0, m1/L1, m2/L2).  Only the Gamma half sphere is stored
  (m = 0 plus every m whose first nonzero component is positive), sorted by
  (|G|^2, m0, m1, m2) so that m = 0 comes first.
* Orbitals: for each orbital (occupied first, then conduction) draw
  x ~ N(0,1) of shape (npw, 2), c(m) = (x0 + i x1) exp(-|G_m|^2/4), c(0) = x0;
  then Gram-Schmidt in index order, twice (as Cholesky QR), with the Gamma
  inner product <f|g> = sum_m w_m Re(conj(f_m) g_m), w_0 = 1, w_m = 2.
* Eigenvalues (Hartree): eps_v = -0.5 (Nocc - v)/Nocc for v = 1..Nocc (HOMO at
  0), eps_c = gap + 0.7 (c - 1)/Nc for c = 1..Nc.  The two slopes differ so the
  lowest transition energies are not exactly degenerate.
* f_xc: a smooth positive density rho0 = (2 Nocc / Omega) e^s / mean(e^s), with
  s(r) a random real combination of the 18 lowest nonzero plane waves
  (|m|^2 <= 2, coefficient 0.2 (N(0,1) + i N(0,1)) on the half space, conjugate
  on the other half), and f_xc = -(1/3) (3/pi)^(1/3) rho0^(-2/3), the
  spin-unpolarised Slater-exchange kernel.  Layout [n0][n1][n2], i2 fastest.
* Trial blocks: X ~ N(0,1) of shape [Nb][Nocc][Nc] from rng(seed + 1000),
  a_v = sum_c X_vc phi_c, each trial scaled so sum_v <a_v|a_v> = 1.  Random
  (not in-span) blocks use the orbital recipe without orthonormalisation.

These choices stand in for the paper's NV- supercells: the 72^3 / Nocc = 128
system has the size of the 63-atom (2x2x2) diamond cell used for the gradient
tests, the 108^3 / Nocc = 432 system that of the 215-atom cell.  A batch of
heterogeneous systems (batch_configs) mixes grids of 48^3 to 96^3 at the same
grid spacing with 32 to 256 occupied orbitals.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    cell: tuple            # (L0, L1, L2) bohr, orthorhombic
    n: tuple               # FFT grid (n0, n1, n2)
    ecut_ry: float
    nocc: int
    ncond: int
    gap: float = 0.15
    alpha: float = 0.25
    c_k: float = 2.0
    v_g0: float = 0.0
    nb: int = 4
    nroots: int = 4
    seed: int = 1


def _cubic(L, n):
    return (float(L),) * 3, (int(n),) * 3


CONFIGS = {
    # plain method, FP64, small enough for the oracle in seconds
    "c1": Config("c1", *_cubic(10.0, 24), ecut_ry=15.0, nocc=8, ncond=8, gap=0.2,
                 nb=4, nroots=4, seed=1),
    # the same system on a 27^3 grid: no aliasing of triple products, so grid
    # quadratures equal continuous integrals (used by the analytic pins)
    "c1p": Config("c1p", *_cubic(10.0, 27), ecut_ry=15.0, nocc=8, ncond=8, gap=0.2,
                  nb=4, nroots=4, seed=1),
    # the benchmark workload: 64-atom-like cell, 72^3 grid, 40 Ry, Nocc = 128
    "c2": Config("c2", *_cubic(13.5, 72), ecut_ry=40.0, nocc=128, ncond=128,
                 gap=0.15, nb=16, nroots=8, seed=2),
    # 216-atom-like cell, 108^3, Nocc = 432 (spin-conserving; spin-flip uses c_k = 0)
    "c3": Config("c3", *_cubic(20.2, 108), ecut_ry=40.0, nocc=432, ncond=432,
                 gap=0.15, nb=32, nroots=16, seed=3),
    # parity cases: several tiles, ragged tails, mixed radices, non-cubic grid
    "p1": Config("p1", *_cubic(11.0, 30), ecut_ry=18.0, nocc=20, ncond=12, gap=0.18,
                 nb=5, nroots=4, seed=11),
    "p2": Config("p2", (9.0, 10.0, 11.5), (24, 27, 32), ecut_ry=14.0, nocc=13,
                 ncond=9, gap=0.2, nb=3, nroots=3, seed=12),
    "p3": Config("p3", *_cubic(13.5, 72), ecut_ry=40.0, nocc=36, ncond=20, gap=0.15,
                 nb=7, nroots=4, seed=13),
    # Nocc = 128 with 16-trial blocks on a small grid (the eight-row-tile
    # contraction at a size the oracle applies in seconds)
    "p5": Config("p5", *_cubic(10.0, 24), ecut_ry=12.0, nocc=128, ncond=16, gap=0.15,
                 nb=16, nroots=4, seed=15),
    # grids of the heterogeneous batch outside the compile-time FFT plans
    # (96 = 2^5 3, 60 = 2^2 3 5) at its spacing and cutoff, few orbitals
    "p6": Config("p6", *_cubic(18.0, 96), ecut_ry=40.0, nocc=20, ncond=12, gap=0.15,
                 nb=4, nroots=2, seed=16),
    "p7": Config("p7", *_cubic(11.25, 60), ecut_ry=40.0, nocc=34, ncond=10, gap=0.15,
                 nb=3, nroots=2, seed=17),
    # the batch's smallest grid (48^3 at its spacing and cutoff) with more than
    # 128 occupied orbitals (row-blocked exchange, ragged last block) and an odd block
    "p8": Config("p8", *_cubic(9.0, 48), ecut_ry=40.0, nocc=140, ncond=8, gap=0.15,
                 nb=5, nroots=2, seed=18),
    # more than 128 occupied orbitals (row-blocked exchange: blocks 64, 64, 16)
    "p4": Config("p4", *_cubic(12.0, 36), ecut_ry=20.0, nocc=144, ncond=24, gap=0.15,
                 nb=3, nroots=3, seed=14),
}


BATCH_GRIDS = (48, 60, 72, 96)


def batch_configs(count: int = 12, seed: int = 4000):
    """Heterogeneous batch of systems: for i < count, a grid n from
    {48, 60, 72, 96} (cubic cell L = 0.1875 n bohr, the 72^3 system's spacing,
    40 Ry), Nocc and Nc uniform in [32, 256], a trial block of 4..32 vectors,
    all drawn from rng(seed); system i is generated with seed 400 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(BATCH_GRIDS))
        nocc = int(rng.integers(32, 257))
        nb = int(rng.integers(4, 33))
        out.append(Config(f"b{i:02d}", *_cubic(0.1875 * n, n), ecut_ry=40.0, nocc=nocc,
                          ncond=nocc, gap=0.15, nb=nb, nroots=min(4, nb), seed=400 + i))
    return out


@dataclasses.dataclass
class System:
    cfg: Config
    cell: np.ndarray       # (3,)
    n: tuple
    mill: np.ndarray       # [npw][3] int32, half sphere, m = 0 first
    c_occ: np.ndarray      # [nocc][npw] complex128
    c_cond: np.ndarray     # [ncond][npw] complex128
    eps_occ: np.ndarray    # [nocc]
    eps_cond: np.ndarray   # [ncond]
    fxc: np.ndarray        # [n0][n1][n2] float64
    alpha: float
    c_k: float
    v_g0: float

    @property
    def npw(self):
        return self.mill.shape[0]

    @property
    def nocc(self):
        return self.c_occ.shape[0]

    @property
    def ncond(self):
        return self.c_cond.shape[0]

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def _g2(mill, cell):
    b = 2.0 * math.pi / np.asarray(cell, dtype=np.float64)
    g = mill.astype(np.float64) * b[None, :]
    return np.einsum("ij,ij->i", g, g)


def half_sphere(cell, ecut_ry, n):
    """Gamma half sphere of Miller indices, m = 0 first, canonical order."""
    cell = np.asarray(cell, dtype=np.float64)
    b = 2.0 * math.pi / cell
    mmax = [int(math.floor(math.sqrt(ecut_ry) / bi)) for bi in b]
    for i in range(3):
        if n[i] <= 2 * mmax[i]:
            raise ValueError(f"grid n[{i}]={n[i]} too small for m_max={mmax[i]}")
    rng = [np.arange(-mm, mm + 1) for mm in mmax]
    m = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    g2 = _g2(m, cell)
    keep = g2 <= ecut_ry * (1.0 + 1e-12)
    m, g2 = m[keep], g2[keep]
    first = np.where(m[:, 0] != 0, m[:, 0], np.where(m[:, 1] != 0, m[:, 1], m[:, 2]))
    half = (first > 0) | np.all(m == 0, axis=1)
    m, g2 = m[half], g2[half]
    key = np.lexsort((m[:, 2], m[:, 1], m[:, 0], np.round(g2, 10)))
    m = m[key]
    assert np.all(m[0] == 0)
    return m.astype(np.int32)


def _weights(npw):
    w = np.full(npw, 2.0)
    w[0] = 1.0
    return w


def gamma_dot(f, g):
    """Gamma-point inner product of half-sphere coefficient vectors (input prep)."""
    w = _weights(f.shape[-1])
    return np.sum(w * (f.real * g.real + f.imag * g.imag), axis=-1)


def _decaying(rng, g2):
    x = rng.standard_normal((g2.shape[0], 2))
    c = (x[:, 0] + 1j * x[:, 1]) * np.exp(-g2 / 4.0)
    c[0] = x[0, 0]
    return c


def _gram_schmidt(c):
    """Gram-Schmidt in index order under the Gamma inner product, done twice.

    Each pass is a Cholesky QR: with the Gram matrix G = L L^T, the rows of
    L^-1 c are the Gram-Schmidt vectors of c in index order (row i combines
    rows 0..i with a positive weight on row i), the same set modified
    Gram-Schmidt produces, up to rounding."""
    sw = np.sqrt(_weights(c.shape[1]))
    for _ in range(2):
        x = np.concatenate([c.real * sw, c.imag * sw], axis=1)
        lo = np.linalg.cholesky(x @ x.T)
        c = scipy.linalg.solve_triangular(lo, c, lower=True)
    c[:, 0] = c[:, 0].real
    return c


def _fxc_field(rng, cfg, n):
    cell = np.asarray(cfg.cell, dtype=np.float64)
    omega = float(np.prod(cell))
    ms = [m for m in half_sphere((1.0, 1.0, 1.0), (2 * math.pi) ** 2 * 2.0 + 1e-9,
                                 (5, 5, 5)) if 0 < int(np.dot(m, m)) <= 2]
    assert len(ms) == 9
    coef = 0.2 * (rng.standard_normal(9) + 1j * rng.standard_normal(9))
    axes = [np.arange(n[i]) * (cell[i] / n[i]) for i in range(3)]
    x, y, z = np.meshgrid(*axes, indexing="ij")
    s = np.zeros(n, dtype=np.float64)
    b = 2.0 * math.pi / cell
    for m, cm in zip(ms, coef):
        ph = b[0] * m[0] * x + b[1] * m[1] * y + b[2] * m[2] * z
        s += 2.0 * (cm.real * np.cos(ph) - cm.imag * np.sin(ph))
    e = np.exp(s)
    rho0 = (2.0 * cfg.nocc / omega) * e / e.mean()
    return -(1.0 / 3.0) * (3.0 / math.pi) ** (1.0 / 3.0) * rho0 ** (-2.0 / 3.0)


def make_system(cfg: Config, **overrides) -> System:
    """Build the seeded synthetic system described in the module docstring."""
    if overrides:
        cfg = dataclasses.replace(cfg, **overrides)
    n = tuple(int(v) for v in cfg.n)
    mill = half_sphere(cfg.cell, cfg.ecut_ry, n)
    g2 = _g2(mill, cfg.cell)
    rng = np.random.default_rng(cfg.seed)
    norb = cfg.nocc + cfg.ncond
    if norb > 2 * mill.shape[0] - 1:
        raise ValueError("more orbitals than real plane-wave degrees of freedom")
    c = np.stack([_decaying(rng, g2) for _ in range(norb)])
    c = _gram_schmidt(c)
    fxc = _fxc_field(rng, cfg, n)
    v = np.arange(1, cfg.nocc + 1, dtype=np.float64)
    eps_occ = -0.5 * (cfg.nocc - v) / cfg.nocc
    cc = np.arange(1, cfg.ncond + 1, dtype=np.float64)
    eps_cond = cfg.gap + 0.7 * (cc - 1.0) / cfg.ncond
    return System(cfg=cfg, cell=np.asarray(cfg.cell, dtype=np.float64), n=n, mill=mill,
                  c_occ=c[:cfg.nocc], c_cond=c[cfg.nocc:], eps_occ=eps_occ,
                  eps_cond=eps_cond, fxc=fxc, alpha=cfg.alpha, c_k=cfg.c_k,
                  v_g0=cfg.v_g0)


def trials_in_span(sys: System, nb: int, seed: int | None = None):
    """Trial block a_v = sum_c X_vc phi_c with sum_v <a_v|a_v> = 1 per trial.

    Returns (a [nb][nocc][npw] complex128, X [nb][nocc][ncond])."""
    seed = sys.cfg.seed if seed is None else seed
    rng = np.random.default_rng(seed + 1000)
    x = rng.standard_normal((nb, sys.nocc, sys.ncond))
    x /= np.sqrt(np.sum(x * x, axis=(1, 2)))[:, None, None]
    xf = x.reshape(-1, sys.ncond)
    # contiguous copies of the real and imaginary parts keep the products on BLAS
    cr = np.ascontiguousarray(sys.c_cond.real)
    ci = np.ascontiguousarray(sys.c_cond.imag)
    a = (xf @ cr + 1j * (xf @ ci)).reshape(nb, sys.nocc, -1)
    return a, x


def trials_random(sys: System, nb: int, seed: int | None = None, offset: int = 2000):
    """Random decaying coefficients (not in the conduction span), unit Gamma norm."""
    seed = sys.cfg.seed if seed is None else seed
    rng = np.random.default_rng(seed + offset)
    g2 = _g2(sys.mill, sys.cell)
    a = np.stack([np.stack([_decaying(rng, g2) for _ in range(sys.nocc)])
                  for _ in range(nb)])
    nrm = np.sqrt(np.sum(gamma_dot(a, a), axis=1))
    return a / nrm[:, None, None]


def plane_wave_pair_system(L=7.0, n=12, m1=(1, 0, 0), ecut_ry=3.0, f0=-0.3,
                           alpha=0.25, c_k=2.0, eps_v=-0.1, eps_c=0.2, v_g0=0.0):
    """Nocc = Nc = 1 with phi_v = sqrt(2/Omega) cos(G1.r), phi_c = sqrt(2/Omega) sin(G1.r),
    and a constant f_xc = f0.  Its single excitation energy has a closed form."""
    n3 = (int(n),) * 3
    mill = half_sphere((L, L, L), ecut_ry, n3)
    idx = [i for i, m in enumerate(mill) if tuple(int(t) for t in m) == tuple(m1)]
    if len(idx) != 1:
        raise ValueError("m1 must be a half-sphere vector inside the cutoff")
    c_occ = np.zeros((1, mill.shape[0]), dtype=np.complex128)
    c_cond = np.zeros_like(c_occ)
    c_occ[0, idx[0]] = 1.0 / math.sqrt(2.0)
    c_cond[0, idx[0]] = -1j / math.sqrt(2.0)
    cfg = Config("pw11", (float(L),) * 3, n3, float(ecut_ry), 1, 1, alpha=alpha,
                 c_k=c_k, v_g0=v_g0, nb=1, nroots=1, seed=0)
    return System(cfg=cfg, cell=np.full(3, float(L)), n=n3, mill=mill, c_occ=c_occ,
                  c_cond=c_cond, eps_occ=np.array([eps_v]), eps_cond=np.array([eps_c]),
                  fxc=np.full(n3, float(f0)), alpha=alpha, c_k=c_k, v_g0=v_g0)
