"""Parity of the HIP Liouville apply with the FP64 oracle (needs an MI355X).

Per-term checks (D, K1e, K1d separately, then all) because the K terms are
small next to D: a K-term bug could hide under a whole-operator tolerance.
Bar: FP64 per-trial relative error <= 1e-10; FP32 <= 2e-5 (FP32 arithmetic
through ~10 rounding steps on O(1) values, with headroom)."""
import numpy as np
import pytest

import oracle
from gen import trials_in_span, trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu

TERMS = {"D": 1, "K1E": 2, "K1D": 4, "ALL": 7}


def _ctx(s, nb, prec="fp64", terms=7):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec, terms=terms)


@pytest.mark.parametrize("cfg", ["c1", "p1", "p2"])
@pytest.mark.parametrize("term", ["D", "K1E", "K1D", "ALL"])
def test_apply_fp64_per_term(systems, cfg, term):
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)          # not in the conduction span: exercises the projection
    say(f"apply fp64 cfg={cfg} term={term} nb={nb}")
    L = _ctx(s, nb, "fp64", TERMS[term])
    got = to_complex(L.apply(a))
    L.close()
    ref = oracle.apply_liouville(s, a, terms=TERMS[term])
    err = rel_err(got, ref)
    say(f"  rel err {err:.3e}")
    assert err <= 1e-10


def test_apply_72cubed_fp64(systems):
    """72^3 grid (compile-time FFT plans), Nocc = 36 (ragged 16-row tiles), Nb = 7."""
    s = systems("p3")
    nb = s.cfg.nb
    a = trials_random(s, nb)
    for term in ("K1D", "ALL"):
        say(f"apply fp64 cfg=p3 term={term} nb={nb}")
        L = _ctx(s, nb, "fp64", TERMS[term])
        got = to_complex(L.apply(a))
        L.close()
        ref = oracle.apply_liouville(s, a, terms=TERMS[term])
        err = rel_err(got, ref)
        say(f"  rel err {err:.3e}")
        assert err <= 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_apply_nocc128_nb16(systems, prec, tol):
    """Nocc = 128, Nb = 16 on a 24^3 grid: the eight-row-tile contraction of
    the benchmark workload, compared element by element."""
    s = systems("p5")
    a = trials_random(s, 16)
    for term in ("K1D", "ALL"):
        say(f"apply {prec} cfg=p5 (Nocc=128, Nb=16) term={term}")
        L = _ctx(s, 16, prec, TERMS[term])
        got = to_complex(L.apply(a))
        L.close()
        err = rel_err(got, oracle.apply_liouville(s, a, terms=TERMS[term]))
        say(f"  rel err {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("cfg,prec,tol,ck", [("p6", "fp32", 2e-5, None),
                                             ("p6", "fp64", 1e-10, 0.0),
                                             ("p7", "fp64", 1e-10, None),
                                             ("p7", "fp32", 2e-5, None),
                                             ("p8", "fp32", 2e-5, None),
                                             ("p8", "fp64", 1e-10, None)])
def test_apply_batch_grids(systems, cfg, prec, tol, ck):
    """The 96^3, 60^3 and 48^3 grids of the heterogeneous batch (a radix-5
    factor on 60^3; 140 occupied orbitals on 48^3, so the exchange runs
    row-blocked with a ragged last block), sampled output rows against the
    oracle (FP64 on 96^3 with c_K = 0, the spin-flip operator; with the
    density response in the next test)."""
    s = systems(cfg) if ck is None else systems(cfg, c_k=ck)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    rows = [0, s.nocc // 2, s.nocc - 1]
    say(f"apply {prec} cfg={cfg} grid={s.n} rows={rows}")
    L = _ctx(s, nb, prec)
    got = to_complex(L.apply(a))[:, rows]
    L.close()
    ref = oracle.apply_liouville(s, a, rows=rows)
    err = rel_err(got, ref)
    say(f"  rel err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("term", ["K1E", "K1D"])
def test_apply_48cubed_blocked_terms_fp32(systems, term):
    """The K terms alone on the 48^3 / Nocc = 140 / Nb = 5 system (sampled
    rows): they are small next to D, so they are checked on their own."""
    s = systems("p8")
    a = trials_random(s, s.cfg.nb)
    rows = [0, 70, 139]
    say(f"apply fp32 cfg=p8 term={term} rows={rows}")
    L = _ctx(s, s.cfg.nb, "fp32", TERMS[term])
    got = to_complex(L.apply(a))[:, rows]
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a, terms=TERMS[term], rows=rows))
    say(f"  rel err {err:.3e}")
    assert err <= 2e-5


@pytest.mark.parametrize("term", ["K1E", "ALL"])
def test_fp64_96_with_response(systems, term):
    """FP64 on the 96^3 grid with the density response: the 96 x 96 FP64 plane
    (147 KB) fits in LDS and the compile-time-plan trial transform keeps the
    density accumulator in registers."""
    s = systems("p6")
    a = trials_random(s, s.cfg.nb)
    rows = [0, s.nocc // 2, s.nocc - 1]
    say(f"apply fp64 cfg=p6 (96^3) term={term} rows={rows}")
    L = _ctx(s, s.cfg.nb, "fp64", TERMS[term])
    got = to_complex(L.apply(a))[:, rows]
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a, terms=TERMS[term], rows=rows))
    say(f"  rel err {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("cfg", ["c1", "p1", "p3"])
def test_apply_fp32(systems, cfg):
    s = systems(cfg)
    nb = s.cfg.nb
    a, _ = trials_in_span(s, nb)
    say(f"apply fp32 cfg={cfg}")
    for term in ("K1E", "K1D", "ALL"):
        L = _ctx(s, nb, "fp32", TERMS[term])
        got = to_complex(L.apply(a))
        L.close()
        ref = oracle.apply_liouville(s, a, terms=TERMS[term])
        err = rel_err(got, ref)
        say(f"  term={term} rel err {err:.3e}")
        assert err <= 2e-5


def test_apply_nb_smaller_than_max_and_odd(systems):
    s = systems("p1")
    a = trials_random(s, 3)
    say("apply nb=3 on a max_nb=6 context, then nb=1")
    L = _ctx(s, 6)
    for nb in (3, 1):
        got = to_complex(L.apply(a[:nb]))
        ref = oracle.apply_liouville(s, a[:nb])
        assert rel_err(got, ref) <= 1e-10
    L.close()


def test_transition_apply_matches_oracle(systems):
    s = systems("p2")
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3, s.nocc, s.ncond))
    say("apply_transition fp64 p2")
    L = _ctx(s, 3)
    got = L.apply_transition(X).cpu().numpy()
    L.close()
    ref = oracle.apply_transition(s, X)
    assert rel_err(got, ref) <= 1e-10


def test_deterministic_bitwise(systems):
    s = systems("p1")
    a = trials_random(s, 5)
    say("determinism fp64 p1")
    L = _ctx(s, 5)
    r1 = L.apply(a).cpu().numpy()
    r2 = L.apply(a).cpu().numpy()
    L.close()
    assert np.array_equal(r1, r2)


def test_v_g0_and_scales(systems):
    s = systems("p2").replace(v_g0=0.9, alpha=0.45, c_k=1.0)
    a = trials_random(s, 2)
    say("v_g0 = 0.9, alpha = 0.45, c_K = 1")
    L = _ctx(s, 2)
    got = to_complex(L.apply(a))
    L.close()
    assert rel_err(got, oracle.apply_liouville(s, a)) <= 1e-10


def test_set_occ_rotation_invariance(systems):
    """K terms with rotated occupied orbitals: L_K(Phi U, A U) = L_K(Phi, A) U."""
    s = systems("p2")
    U, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((s.nocc, s.nocc)))
    a = trials_random(s, 2)
    say("set_occ rotation invariance p2")
    L = _ctx(s, 2, terms=6)
    base = to_complex(L.apply(a))
    L.set_occ(U.T @ s.c_occ)
    rot = to_complex(L.apply(np.einsum("vn,bvm->bnm", U, a)))
    L.close()
    assert rel_err(rot, np.einsum("vn,bvm->bnm", U, base)) <= 1e-10


def test_davidson_c1_matches_dense(systems):
    s = systems("c1")
    n = s.nocc * s.ncond
    M = oracle.apply_transition(s, np.eye(n).reshape(n, s.nocc, s.ncond)).reshape(n, n)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    say("davidson fp64 c1")
    L = _ctx(s, 4)
    omega, x, resid, nit, st = L.davidson(4, 4, tol=1e-8, max_iter=100)
    say(f"  omega={omega} resid={resid} iters={nit} status={st}")
    assert st == 0
    assert np.all(resid <= 1e-8)
    assert np.max(np.abs(omega - ev[:4]) / np.abs(ev[:4])) <= 1e-10
    xc = to_complex(x)
    nrm = oracle.gamma_inner(xc, xc).sum(axis=1)
    assert np.abs(nrm - 1).max() < 1e-10
    # eigenvector check through the oracle: L x = omega x
    lx = oracle.apply_liouville(s, xc)
    assert rel_err(lx, omega[:, None, None] * xc) < 1e-7
    L.close()


def test_davidson_fp32_within_1mev(systems):
    s = systems("c1")
    n = s.nocc * s.ncond
    M = oracle.apply_transition(s, np.eye(n).reshape(n, s.nocc, s.ncond)).reshape(n, n)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    say("davidson fp32 c1")
    L = _ctx(s, 4, "fp32")
    omega, x, resid, nit, st = L.davidson(4, 4, tol=1e-5, max_iter=100)
    L.close()
    say(f"  |d omega| = {np.abs(omega - ev[:4]).max():.3e} Ha")
    assert np.abs(omega - ev[:4]).max() <= 3.674932e-5


def test_error_codes(systems):
    from paper_2309_03513_amd import WtdError
    s = systems("c1")
    L = _ctx(s, 2)
    a = trials_random(s, 3)
    say("error codes")
    with pytest.raises(WtdError) as e:
        L.apply(a)                      # nb = 3 > max_nb = 2
    assert e.value.status == -2
    with pytest.raises(WtdError) as e:
        L.apply_bwd(a, a)               # nb = 3 > max_nb = 2
    assert e.value.status == -2
    with pytest.raises(WtdError) as e:
        L.davidson(3, 2)                # nroots > nb
    assert e.value.status == -2
    om, x, r, nit, st = L.davidson(2, 2, tol=1e-14, max_iter=1)
    assert st == 1                      # WTD_NOT_CONVERGED is a warning
    L.close()


@pytest.mark.parametrize("cfg,prec,tol", [("c1", "fp64", 1e-10), ("p1", "fp64", 1e-10),
                                          ("p5", "fp64", 1e-10), ("c1", "fp32", 2e-5),
                                          ("p5", "fp32", 2e-5)])
def test_apply_stress_per_term(systems, cfg, prec, tol):
    """alpha = 25, c_K = 200: the response and exchange terms outweigh D, so a
    mistake in either shows at the whole-operator scale too.  Per term and
    whole, element by element (the bound covers max |got - ref| / max |ref| as
    well as the relative Frobenius norm of each trial)."""
    s = systems(cfg, alpha=25.0, c_k=200.0)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    for term in ("K1E", "K1D", "ALL"):
        L = _ctx(s, nb, prec, TERMS[term])
        got = to_complex(L.apply(a))
        L.close()
        ref = oracle.apply_liouville(s, a, terms=TERMS[term])
        err = rel_err(got, ref)
        say(f"stress alpha=25 c_K=200 cfg={cfg} {prec} term={term}: err {err:.3e}")
        assert err <= tol


def test_apply_fp32_with_g0_kernel(systems):
    """A Coulomb kernel value at G = 0 in the FP32 path: the apply matches the
    oracle and the lowest roots move by -alpha v_g0 / Omega (the closed form of
    the G = 0 term for in-span trials)."""
    s = systems("c1", v_g0=0.9)
    s0 = systems("c1")
    nb = s.cfg.nb
    a, _ = trials_in_span(s, nb)
    say("apply fp32 c1 v_g0 = 0.9")
    L = _ctx(s, nb, "fp32")
    got = to_complex(L.apply(a))
    err = rel_err(got, oracle.apply_liouville(s, a))
    om, _, _, _, st = L.davidson(4, 4, tol=1e-5, want_x=False)
    L.close()
    L0 = _ctx(s0, nb, "fp32")
    om0, _, _, _, st0 = L0.davidson(4, 4, tol=1e-5, want_x=False)
    L0.close()
    shift = -s.alpha * 0.9 / float(np.prod(s.cell))
    say(f"  rel err {err:.3e}; root shift {np.max(np.abs(om - om0 - shift)):.3e} off the closed form")
    assert err <= 2e-5
    assert st == 0 and st0 == 0
    assert np.max(np.abs(om - om0 - shift)) <= 3.674932e-5
