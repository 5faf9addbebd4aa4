"""Parity of the full operator D + K1e - K1d + K2e - K2d (wtd_apply_full) and of
the Z-vector CG solve (wtd_solve_zvector) with the FP64 oracle (needs an MI355X).

Per term as for the TDA operator: K2e and K2d alone, then the full operator;
FP64 per-trial relative error <= 1e-10, FP32 <= 2e-5.  K2d's pair fields are
processed in row chunks of the pair buffer, so the cases cover several chunks,
an odd Nocc (chunks of an even number of rows), the row-blocked exchange and
the eight-row-tile contraction size (Nocc = 128, Nb = 16)."""
import numpy as np
import pytest

import oracle
from gen import trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu

K2 = oracle.TERM_K2E | oracle.TERM_K2D
TERMS = {"K2E": oracle.TERM_K2E, "K2D": oracle.TERM_K2D, "FULL": oracle.TERM_FULL}


def _ctx(s, nb, prec, terms):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec, terms=terms)


@pytest.mark.parametrize("cfg", ["c1", "p1", "p2"])
@pytest.mark.parametrize("term", ["K2E", "K2D", "FULL"])
def test_full_operator_fp64_per_term(systems, cfg, term):
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    say(f"apply_full fp64 cfg={cfg} term={term} nb={nb}")
    L = _ctx(s, nb, "fp64", TERMS[term])
    got = to_complex(L.apply_full(a))
    L.close()
    ref = oracle.apply_liouville(s, a, terms=TERMS[term])
    err = rel_err(got, ref)
    say(f"  rel err {err:.3e}")
    assert err <= 1e-10


def test_tda_entry_point_ignores_k2_terms(systems):
    s = systems("p1")
    a = trials_random(s, 2)
    L = _ctx(s, 2, "fp64", oracle.TERM_FULL)
    got = to_complex(L.apply(a))
    L.close()
    assert rel_err(got, oracle.apply_liouville(s, a)) <= 1e-10


@pytest.mark.parametrize("cfg,prec,tol,rows", [("p3", "fp64", 1e-10, [0, 17, 35]),
                                               ("p3", "fp32", 2e-5, [0, 17, 35]),
                                               ("p5", "fp64", 1e-10, [0, 77, 127]),
                                               ("p5", "fp32", 2e-5, [0, 77, 127])])
def test_full_operator_sampled_rows(systems, cfg, prec, tol, rows):
    """72^3 grid with Nocc = 36 (the fused K2d inverse pass and contraction);
    Nocc = 128 with Nb = 16 (two row chunks of K2d pairs)."""
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    say(f"apply_full {prec} cfg={cfg} rows={rows}")
    L = _ctx(s, nb, prec, oracle.TERM_FULL)
    got = to_complex(L.apply_full(a))[:, rows]
    L.close()
    ref = oracle.apply_liouville(s, a, terms=oracle.TERM_FULL, rows=rows)
    err = rel_err(got, ref)
    say(f"  rel err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("cfg,rb,rows", [("p1", "16", None), ("p4", "0", [0, 71, 143])])
def test_full_operator_row_blocked(systems, monkeypatch, cfg, rb, rows):
    """Row-blocked exchange: forced blocks of 16 rows, and Nocc = 144."""
    if rb != "0":
        monkeypatch.setenv("WTD_ROW_BLOCK", rb)
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    say(f"apply_full fp64 row-blocked cfg={cfg} rb={rb}")
    L = _ctx(s, nb, "fp64", oracle.TERM_FULL)
    got = to_complex(L.apply_full(a))
    L.close()
    if rows is not None:
        got = got[:, rows]
    ref = oracle.apply_liouville(s, a, terms=oracle.TERM_FULL, rows=rows)
    err = rel_err(got, ref)
    say(f"  rel err {err:.3e}")
    assert err <= 1e-10


def _rhs(s, nrhs, seed):
    # right-hand sides of different sizes, so that with lambda_thr > 0 the
    # systems cross the threshold at different iterations
    nocc, nc = s.c_occ.shape[0], s.c_cond.shape[0]
    X = np.random.default_rng(seed).standard_normal((nrhs, nocc, nc))
    X *= (0.3 ** np.arange(nrhs))[:, None, None]
    return X, np.einsum("bvc,cm->bvm", X, s.c_cond)


@pytest.mark.parametrize("cfg,prec,nrhs,lam,tol", [("c1", "fp64", 2, 0.0, 1e-9),
                                                   ("c1", "fp64", 1, 1e-3, 1e-9),
                                                   ("c1", "fp64", 3, 1e-3, 1e-9),
                                                   ("p2", "fp64", 2, 3e-3, 1e-9),
                                                   ("p2", "fp64", 3, 0.0, 1e-9),
                                                   ("c1", "fp32", 2, 0.0, 1e-4)])
def test_zvector_cg_matches_oracle(systems, cfg, prec, nrhs, lam, tol):
    s = systems(cfg)
    X, U = _rhs(s, nrhs, 21)
    lam_abs = lam * float(np.linalg.norm(X))
    say(f"zvector CG {prec} cfg={cfg} nrhs={nrhs} lambda_thr={lam_abs:.2e}")
    L = _ctx(s, nrhs, prec, oracle.TERM_FULL)
    Z, res, it, nex, st = L.solve_zvector(U, tol=1e-10 if prec == "fp64" else 1e-7,
                                          max_iter=200, lambda_thr=lam_abs)
    L.close()
    assert st == 0
    Zo, reso, ito, nexo = oracle.solve_zvector_transition(
        s, X, tol=1e-10 if prec == "fp64" else 1e-7, max_iter=200, lambda_thr=lam_abs)
    ref = np.einsum("bvc,cm->bvm", Zo, s.c_cond)
    err = rel_err(to_complex(Z), ref)
    say(f"  iterations {it} (oracle {ito}), exact applies {nex} (oracle {nexo}), rel err {err:.3e}")
    assert err <= tol
    assert abs(it - ito) <= 1
    if lam > 0.0:
        assert 0 < nex < it and abs(nex - nexo) <= 1
    else:
        assert nex == it
