"""Pins of the CPU oracle against routes other than itself (no GPU).

Each test reaches a quantity the oracle computes by an independent route, or
checks a property the paper or the mathematics fixes, so that a dropped term, a
wrong sign or index, or a transposed operand in the oracle fails one of them.
"""
import math

import numpy as np
import pytest

import oracle
from gen import CONFIGS, Config, make_system, plane_wave_pair_system, trials_in_span, trials_random
from tests import pinlib

ALL = oracle.TERM_ALL
K_ONLY = oracle.TERM_K1E | oracle.TERM_K1D


def _dense(s, terms=ALL):
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    n = nocc * nc
    M = oracle.apply_transition(s, np.eye(n).reshape(n, nocc, nc), terms=terms)
    return M.reshape(n, n).T


def _tiny(name="tiny", cell=(5.0, 5.5, 6.0), n=(8, 9, 10), ecut=4.0, nocc=3, ncond=4, seed=7):
    return make_system(Config(name, tuple(cell), tuple(n), ecut, nocc, ncond, gap=0.2,
                              alpha=0.3, c_k=2.0, seed=seed))


# ---------------------------------------------------------------- transforms (Sec. 2, Gamma point)
def test_real_space_matches_direct_dft():
    s = _tiny()
    ref = pinlib.direct_real_space(s.c_occ, s.mill, s.cell, s.n)
    got = oracle.real_space(s.c_occ, s.mill, s.cell, s.n)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_coefficients_match_direct_dft():
    s = _tiny()
    rng = np.random.default_rng(3)
    f = rng.standard_normal((2,) + s.n)
    ref = pinlib.direct_coefficients(f, s.mill, s.cell)
    got = oracle.coefficients(f, s.mill, s.cell)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_round_trip_and_gamma_inner_is_quadrature():
    s = _tiny()
    phi = oracle.real_space(s.c_occ, s.mill, s.cell, s.n)
    back = oracle.coefficients(phi, s.mill, s.cell)
    assert np.abs(back - s.c_occ).max() < 1e-13
    omega, nr = float(np.prod(s.cell)), int(np.prod(s.n))
    quad = (omega / nr) * phi.reshape(3, -1) @ phi.reshape(3, -1).T
    gi = oracle.gamma_inner(s.c_occ[:, None, :], s.c_occ[None, :, :])
    assert np.abs(quad - gi).max() < 1e-13
    assert np.abs(gi - np.eye(3)).max() < 1e-13


def test_gamma_overlap_is_quadrature():
    """<f_i|g_j> of two unrelated coefficient sets equals the grid quadrature
    (Omega/N_r) sum_j f(r_j) g(r_j) of their real-space fields."""
    s = _tiny()
    rng = np.random.default_rng(41)
    npw = s.mill.shape[0]
    f = rng.standard_normal((4, npw)) + 1j * rng.standard_normal((4, npw))
    g = rng.standard_normal((5, npw)) + 1j * rng.standard_normal((5, npw))
    f[:, 0] = f[:, 0].real
    g[:, 0] = g[:, 0].real
    F = oracle.real_space(f, s.mill, s.cell, s.n).reshape(4, -1)
    G = oracle.real_space(g, s.mill, s.cell, s.n).reshape(5, -1)
    omega, nr = float(np.prod(s.cell)), int(np.prod(s.n))
    quad = (omega / nr) * F @ G.T
    ov = oracle.gamma_overlap(f, g)
    assert ov.shape == (4, 5)
    assert np.abs(quad - ov).max() <= 1e-12 * np.abs(quad).max()


# ---------------------------------------------------------------- Coulomb kernel / Poisson
@pytest.mark.parametrize("v_g0", [0.0, 0.37])
def test_poisson_matches_realspace_coulomb_sum(v_g0):
    cell, n = (4.0, 4.5, 5.0), (6, 7, 8)
    rng = np.random.default_rng(5)
    rho = rng.standard_normal(n)
    ref = pinlib.realspace_poisson(rho, cell, n, v_g0)
    got = oracle.poisson(rho, oracle.coulomb_kernel(cell, n, v_g0))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("L,m1", [(7.0, (1, 0, 0)), (8.5, (1, 1, 0)), (9.0, (2, 1, -1))])
def test_plane_wave_pair_integrals_closed_form(L, m1):
    """phi_v = sqrt(2/Omega) cos(G1.r), phi_c = sqrt(2/Omega) sin(G1.r):
    (cv|cv) = pi/(2 Omega |G1|^2), (cc|vv) = -pi/(2 Omega |G1|^2) (G = 0 dropped)."""
    s = plane_wave_pair_system(L=L, n=16, m1=m1, ecut_ry=(2 * math.pi / L) ** 2 * 6.5)
    omega = L ** 3
    g1sq = (2 * math.pi / L) ** 2 * sum(t * t for t in m1)
    phv = oracle.real_space(s.c_occ[0], s.mill, s.cell, s.n)
    phc = oracle.real_space(s.c_cond[0], s.mill, s.cell, s.n)
    pts = pinlib.grid_points(s.cell, s.n)
    g1 = np.asarray(m1) * (2 * math.pi / L)
    assert np.allclose(phv.ravel(), math.sqrt(2 / omega) * np.cos(pts @ g1), atol=1e-14)
    assert np.allclose(phc.ravel(), math.sqrt(2 / omega) * np.sin(pts @ g1), atol=1e-14)
    kern = oracle.coulomb_kernel(s.cell, s.n, 0.0)
    w = omega / np.prod(s.n)
    cvcv = w * np.sum(phc * phv * oracle.poisson(phc * phv, kern))
    ccvv = w * np.sum(phc * phc * oracle.poisson(phv * phv, kern))
    ref = math.pi / (2 * omega * g1sq)
    assert abs(cvcv - ref) <= 1e-14 * ref * 10
    assert abs(ccvv + ref) <= 1e-14 * ref * 10


# ---------------------------------------------------------------- the whole operator, closed form
@pytest.mark.parametrize("alpha,c_k,f0", [(0.25, 2.0, -0.3), (0.0, 2.0, 0.1), (0.4, 0.0, -0.2),
                                          (0.25, 1.0, 0.0)])
def test_one_by_one_excitation_closed_form(alpha, c_k, f0):
    """omega = de + (c_K + alpha) pi/(2 Omega |G1|^2) + c_K f0/(2 Omega)."""
    L, m1 = 7.5, (1, 1, 0)
    s = plane_wave_pair_system(L=L, n=14, m1=m1, ecut_ry=(2 * math.pi / L) ** 2 * 3.5,
                               f0=f0, alpha=alpha, c_k=c_k)
    omega = L ** 3
    g1sq = (2 * math.pi / L) ** 2 * 2
    de = s.eps_cond[0] - s.eps_occ[0]
    ref = de + (c_k + alpha) * math.pi / (2 * omega * g1sq) + c_k * f0 / (2 * omega)
    la = oracle.apply_liouville(s, s.c_cond[None, :, :])
    assert np.abs(la[0, 0] - ref * s.c_cond[0]).max() < 1e-15
    w = oracle.gamma_inner(s.c_cond[0], la[0, 0])
    assert abs(w - ref) < 1e-14


# ---------------------------------------------------------------- Casida assembly without FFTs
@pytest.mark.parametrize("alpha,c_k,v_g0", [(0.25, 2.0, 0.0), (0.0, 2.0, 0.0), (0.6, 1.0, 0.8)])
def test_dense_operator_matches_fft_free_casida(systems, alpha, c_k, v_g0):
    s = systems("c1p").replace(alpha=alpha, c_k=c_k, v_g0=v_g0)
    ref = pinlib.casida_matrix(s)
    got = _dense(s)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- symmetries and reductions
def test_hermitian_in_gamma_inner_product(systems):
    s = systems("p2")
    A = trials_random(s, 3)
    B = trials_random(s, 3, offset=3000)
    lhs = np.sum(oracle.gamma_inner(B, oracle.apply_liouville(s, A)))
    rhs = np.sum(oracle.gamma_inner(oracle.apply_liouville(s, B), A))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1e-3)


def test_exchange_and_response_invariant_under_occupied_rotation(systems):
    """K1e and K1d are invariant under a unitary rotation of the occupied orbitals
    (Sec. 3.2, Eq. trunc): L_K(Phi U, A U) = L_K(Phi, A) U."""
    s = systems("p2")
    nocc = s.nocc
    A = trials_random(s, 2)
    U, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((nocc, nocc)))
    occ_r = U.T @ s.c_occ
    A_r = np.einsum("vn,bvm->bnm", U, A)
    lhs = oracle.apply_liouville(s, A_r, terms=K_ONLY, occ=occ_r)
    rhs = np.einsum("vn,bvm->bnm", U, oracle.apply_liouville(s, A, terms=K_ONLY))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_each_term_breaks_rotation_covariance_only_through_D(systems):
    """Sanity of the check above: with D included the rotation changes the result."""
    s = systems("p2")
    A = trials_random(s, 1)
    U, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((s.nocc, s.nocc)))
    lhs = oracle.apply_liouville(s, np.einsum("vn,bvm->bnm", U, A), occ=U.T @ s.c_occ)
    rhs = np.einsum("vn,bvm->bnm", U, oracle.apply_liouville(s, A))
    assert np.abs(lhs - rhs).max() > 1e-6


def test_d_only_spectrum_is_transition_energies(systems):
    s = systems("c1").replace(alpha=0.0, c_k=0.0)
    ev = np.linalg.eigvalsh(_dense(s))
    de = np.sort((s.eps_cond[None, :] - s.eps_occ[:, None]).ravel())
    assert np.abs(ev - de).max() < 1e-14


def test_alpha_zero_drops_exchange(systems):
    s = systems("c1")
    full = _dense(s.replace(alpha=0.0))
    no_k1d = _dense(s, terms=oracle.TERM_D | oracle.TERM_K1E)
    assert np.abs(full - no_k1d).max() < 1e-15


def test_coulomb_g0_shifts_every_root(systems):
    """v_g0 != 0 changes only tau_vv by v_g0/Omega: every omega shifts by -alpha v_g0/Omega."""
    s = systems("c1")
    v_g0 = 1.7
    e0 = np.linalg.eigvalsh(_dense(s))
    e1 = np.linalg.eigvalsh(_dense(s.replace(v_g0=v_g0)))
    shift = -s.alpha * v_g0 / float(np.prod(s.cell))
    assert np.abs(e1 - e0 - shift).max() < 1e-13


def test_projector_readings_agree_for_complete_basis():
    """Nocc + Nc = all real degrees of freedom: sum_c |c><c| = 1 - sum_v |v><v|."""
    s = make_system(Config("cb", (6.0, 6.0, 6.0), (8, 8, 8), 1.2, 3, 4, gap=0.2, alpha=0.3,
                           c_k=2.0, seed=21))
    assert 2 * s.npw - 1 == 7
    A = trials_random(s, 2)
    span = oracle.apply_liouville(s, A, projector="span")
    comp = oracle.apply_liouville(s, A, projector="complement")
    assert np.abs(span - comp).max() < 1e-13


def test_rows_subset_matches_full(systems):
    s = systems("p1")
    a, _ = trials_in_span(s, 2)
    full = oracle.apply_liouville(s, a)
    part = oracle.apply_liouville(s, a, rows=[0, 7, 19])
    assert np.abs(part - full[:, [0, 7, 19]]).max() < 1e-15


# ---------------------------------------------------------------- Davidson (Sec. 4)
def test_davidson_matches_dense_eigh(systems):
    s = systems("c1")
    ev = np.linalg.eigvalsh(_dense(s))
    th, X, rn, it, ok = oracle.davidson_transition(s, nroots=4, nb=4, tol=1e-8)
    assert ok and np.all(rn <= 1e-8)
    assert np.abs(th - ev[:4]).max() <= 1e-10 * np.abs(ev[:4]).max()
    assert np.abs(np.linalg.norm(X, axis=0) - 1.0).max() < 1e-12


def test_davidson_restart_path(systems):
    s = systems("c1")
    ev = np.linalg.eigvalsh(_dense(s))
    th, X, rn, it, ok = oracle.davidson_transition(s, nroots=3, nb=3, tol=1e-9, max_sub=6)
    assert ok
    assert np.abs(th - ev[:3]).max() <= 1e-10


def test_rayleigh_ritz_certificate_against_eigh():
    """The Rayleigh-Ritz certificate on a dense symmetric matrix with a known
    spectrum: Ritz values equal eigvalsh of the projected matrix, and the
    Weinstein and Kato-Temple bounds hold, and are tight enough to matter, for
    perturbed eigenvectors."""
    from tests.certify import rayleigh_ritz
    rng = np.random.default_rng(41)
    n, k = 40, 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = 0.1 + 0.1 * np.arange(n) + rng.uniform(-0.02, 0.02, n)
    A = (Q * ev) @ Q.T
    A = 0.5 * (A + A.T)
    V = Q[:, :k] + 1e-3 * rng.standard_normal((n, k))
    theta, Y, rn, kt = rayleigh_ritz(lambda B: A @ B, V)
    P, _ = np.linalg.qr(V)
    assert np.abs(theta - np.linalg.eigvalsh(P.T @ A @ P)).max() <= 1e-13
    assert np.abs(Y.T @ Y - np.eye(k)).max() <= 1e-13
    err = np.abs(theta - ev[:k])
    assert np.all(err <= rn + 1e-14)
    assert all(err[i] <= kt[i] + 1e-14 for i in range(k - 1)) and kt[-1] is None
    # the perturbation is visible and the quadratic bound is well below the linear one
    assert err.max() > 1e-8 and all(kt[i] < 0.2 * rn[i] for i in range(k - 1))


def test_benchmark_kato_temple_matches_certificate():
    """The benchmark's Kato-Temple bounds of Davidson roots (from Ritz values and
    residual norms alone) equal the certificate's on the same Ritz pairs."""
    import bench
    from tests.certify import rayleigh_ritz
    rng = np.random.default_rng(47)
    n, k = 30, 5
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * (0.1 + 0.1 * np.arange(n))) @ Q.T
    A = 0.5 * (A + A.T)
    theta, _, rn, kt = rayleigh_ritz(lambda B: A @ B, Q[:, :k] + 1e-3 * rng.standard_normal((n, k)))
    got = bench.kato_temple(theta, rn)
    assert got[-1] is None and kt[-1] is None
    assert np.allclose(got[:-1], kt[:-1], rtol=1e-14, atol=0.0)


def test_rayleigh_ritz_on_oracle_operator_bounds_the_dense_roots(systems):
    """The certificate with the oracle's operator as the matvec (as the GPU
    eigenvector checks use it) on perturbed eigenvectors of C1's dense matrix."""
    from tests.certify import rayleigh_ritz, transition_matvec
    s = systems("c1")
    ev, W = np.linalg.eigh(_dense(s))
    rng = np.random.default_rng(43)
    k = 5
    V = W[:, :k] + 1e-4 * rng.standard_normal((W.shape[0], k))
    theta, _, rn, kt = rayleigh_ritz(transition_matvec(s), V)
    err = np.abs(theta - ev[:k])
    assert np.all(err <= rn + 1e-13)
    assert all(err[i] <= kt[i] + 1e-13 for i in range(k - 1))
    assert all(kt[i] < 0.5 * rn[i] for i in range(k - 1))


def test_davidson_exhausted_basis_reports_its_iteration():
    """With a tolerance below rounding, the basis of a 12 x 12 problem fills up
    after three blocks of 4; every later correction is dropped, so the run
    stops unconverged at that iteration (not at max_iter) with the exact
    spectrum of the matrix."""
    rng = np.random.default_rng(31)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    ev = np.sort(rng.uniform(0.1, 2.0, 12))
    A = (Q * ev) @ Q.T
    A = 0.5 * (A + A.T)
    th, X, rn, it, ok = oracle.davidson(lambda V: A @ V, np.diag(A), nroots=4, nb=4, tol=0.0,
                                        max_iter=50)
    assert not ok
    assert 3 <= it <= 4
    assert np.abs(th - ev[:4]).max() <= 1e-12
    assert np.all(rn <= 1e-12)
