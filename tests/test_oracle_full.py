"""Pins of the oracle's full operator D + K1e - K1d + K2e - K2d (Eq. z-v-eq)
and of its conjugate-gradient Z-vector solve with the inexact Krylov switch
(Sec. 3.3), against routes other than the oracle itself (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from gen import plane_wave_pair_system, trials_random
from tests import pinlib

FULL = oracle.TERM_FULL
APPROX = oracle.TERM_FULL & ~oracle.TERM_K2D


def _dense(s, terms):
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    n = nocc * nc
    M = oracle.apply_transition(s, np.eye(n).reshape(n, nocc, nc), terms=terms)
    return M.reshape(n, n).T


@pytest.mark.parametrize("alpha,c_k,f0", [(0.25, 2.0, -0.3), (0.4, 0.0, -0.2), (0.0, 1.0, 0.1)])
def test_one_by_one_full_operator_closed_form(alpha, c_k, f0):
    """Plane-wave pair phi_v ~ cos(G1.r), phi_c ~ sin(G1.r): K2e equals K1e,
    c_K (pi/(2 Omega |G1|^2) + f0/(2 Omega)); K2d is +alpha pi/(2 Omega |G1|^2),
    the opposite of K1d, so the full operator is de + 2 K1e."""
    L, m1 = 7.5, (1, 1, 0)
    s = plane_wave_pair_system(L=L, n=14, m1=m1, ecut_ry=(2 * math.pi / L) ** 2 * 3.5,
                               f0=f0, alpha=alpha, c_k=c_k)
    omega = L ** 3
    g1sq = (2 * math.pi / L) ** 2 * 2
    de = s.eps_cond[0] - s.eps_occ[0]
    ke = c_k * (math.pi / (2 * omega * g1sq) + f0 / (2 * omega))
    kd2 = alpha * math.pi / (2 * omega * g1sq)
    a = s.c_cond[None, :, :]
    for terms, ref in [(FULL, de + 2 * ke), (oracle.TERM_K2E, ke), (oracle.TERM_K2D, -kd2),
                       (APPROX, de + 2 * ke + kd2)]:
        la = oracle.apply_liouville(s, a, terms=terms)
        w = oracle.gamma_inner(s.c_cond[0], la[0, 0])
        assert abs(w - ref) < 1e-14, (terms, w, ref)


@pytest.mark.parametrize("alpha,c_k,v_g0", [(0.25, 2.0, 0.0), (0.6, 1.0, 0.8), (0.3, 0.0, 0.0)])
def test_full_operator_matches_fft_free_casida(systems, alpha, c_k, v_g0):
    """Dense full operator = A + B with B assembled from direct convolutions."""
    s = systems("c1p").replace(alpha=alpha, c_k=c_k, v_g0=v_g0)
    ref = pinlib.casida_matrix(s) + pinlib.casida_b_matrix(s)
    got = _dense(s, FULL)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # K2 terms alone
    got_b = _dense(s, oracle.TERM_K2E | oracle.TERM_K2D)
    assert np.abs(got_b - pinlib.casida_b_matrix(s)).max() <= 1e-12 * np.abs(ref).max()


def test_k2_terms_invariant_under_occupied_rotation(systems):
    """K2e, K2d (ΦU, AU) = K2e, K2d (Φ, A) U for an orthogonal U (Eq. trunc's
    invariance carries over: both are sums over the occupied index)."""
    s = systems("p2")
    a = trials_random(s, 2)
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((s.nocc, s.nocc)))
    terms = oracle.TERM_K2E | oracle.TERM_K2D
    ref = np.einsum("bvm,vu->bum", oracle.apply_liouville(s, a, terms=terms), U)
    got = oracle.apply_liouville(s, np.einsum("bvm,vu->bum", a, U), terms=terms,
                                 occ=U.T @ s.c_occ)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_full_operator_rows_subset(systems):
    s = systems("c1")
    a = trials_random(s, 2)
    full = oracle.apply_liouville(s, a, terms=FULL)
    part = oracle.apply_liouville(s, a, terms=FULL, rows=[1, 5])
    assert np.abs(part - full[:, [1, 5]]).max() <= 1e-14 * np.abs(full).max()


def test_cg_matches_dense_solve(systems):
    s = systems("c1")
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    M = _dense(s, FULL)
    assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0          # the CG needs a positive operator
    rng = np.random.default_rng(9)
    U = rng.standard_normal((2, nocc, nc))
    Z, res, its, nex = oracle.solve_zvector_transition(s, U, tol=1e-12, max_iter=200)
    for k in range(2):
        ref = np.linalg.solve(M, U[k].ravel())
        assert np.abs(Z[k].ravel() - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(res <= 1e-12) and nex == its


def test_single_cg_matches_block_solve(systems):
    """The block solve with one right-hand side takes the steps of cg_inexact."""
    s = systems("c1")
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    U = np.random.default_rng(12).standard_normal((1, nocc, nc))
    thr = 1e-3 * np.linalg.norm(U)
    Z, res, its, nex = oracle.solve_zvector_transition(s, U, tol=1e-10, lambda_thr=thr)

    def mv(terms):
        return lambda x: oracle.apply_transition(s, x.reshape(1, nocc, nc), terms=terms).ravel()

    z, rn, it, ne = oracle.cg_inexact(mv(FULL), mv(APPROX), U[0], 1e-10, 200, thr)
    assert (it, ne) == (its, nex)
    assert np.abs(z - Z[0].ravel()).max() <= 1e-13 * np.abs(z).max()


def test_inexact_switch(systems):
    """lambda_thr above the first residual: every apply is the approximate
    operator, so Z solves (L - K2d) Z = U; a middle threshold switches once."""
    s = systems("c1")
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    Ma = _dense(s, APPROX)
    M = _dense(s, FULL)
    rng = np.random.default_rng(10)
    U = rng.standard_normal((1, nocc, nc))
    Z, res, its, nex = oracle.solve_zvector_transition(s, U, tol=1e-12, lambda_thr=1e6)
    assert nex == 0
    ref = np.linalg.solve(Ma, U[0].ravel())
    assert np.abs(Z[0].ravel() - ref).max() <= 1e-10 * np.abs(ref).max()
    thr = 1e-3 * np.linalg.norm(U)
    Z, res, its, nex = oracle.solve_zvector_transition(s, U, tol=1e-12, lambda_thr=thr)
    assert 0 < nex < its
    exact = np.linalg.solve(M, U[0].ravel())
    err = np.linalg.norm(Z[0].ravel() - exact) / np.linalg.norm(exact)
    # the approximate phase corrects a residual of size ~thr with an operator
    # that differs by K2d: the error stays at the size of thr relative to U
    assert err <= 10 * thr / np.linalg.norm(U)


def test_inexact_switch_is_per_system(systems):
    """Two right-hand sides whose first residuals lie on either side of
    lambda_thr: the small one is solved with the approximate operator from the
    start (so it solves (L - K2d) Z = U to tol), the large one starts exact and
    switches later (error of the size of thr), as two separate CG solves do."""
    s = systems("c1")
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    Ma = _dense(s, APPROX)
    M = _dense(s, FULL)
    rng = np.random.default_rng(13)
    U = rng.standard_normal((2, nocc, nc))
    U[1] *= 1e-4
    thr = 1e-2 * np.linalg.norm(U[0])
    assert np.linalg.norm(U[1]) < thr < np.linalg.norm(U[0])
    Z, res, its, nex = oracle.solve_zvector_transition(s, U, tol=1e-13, lambda_thr=thr)
    ref_a = np.linalg.solve(Ma, U[1].ravel())
    assert np.abs(Z[1].ravel() - ref_a).max() <= 1e-9 * np.abs(ref_a).max()
    exact = np.linalg.solve(M, U[0].ravel())
    err = np.linalg.norm(Z[0].ravel() - exact) / np.linalg.norm(exact)
    assert 1e-14 < err <= 10 * thr / np.linalg.norm(U[0])
    assert 0 < nex < its
