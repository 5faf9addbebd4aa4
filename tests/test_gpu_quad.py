"""The register-quad plane kernels (lines held by quads of lanes, one LDS
transpose per 2D FFT), which the library takes where a complex plane does not
fit in LDS (FP64 108 x 108) and everywhere else they apply when
WTD_QUAD_PLANES=1 is set at context creation: applies against the oracle on
grids of 24, 48, 72 and 96 points, the Davidson roots against the stored
oracle roots, and the 108^3 FP64 operator in the 108^3 parity file."""
import json
import os

import numpy as np
import pytest

import oracle
from gen import trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu

TERMS = {"D": 1, "K1E": 2, "K1D": 4, "ALL": 7}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ctx(s, nb, prec, terms=7):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec, terms=terms)


@pytest.mark.parametrize("cfg,prec,term,tol", [("p5", "fp64", "ALL", 1e-10),
                                               ("p5", "fp64", "K1D", 1e-10),
                                               ("p5", "fp32", "ALL", 2e-5),
                                               ("p3", "fp64", "K1E", 1e-10),
                                               ("p3", "fp64", "ALL", 1e-10),
                                               ("p3", "fp32", "K1D", 2e-5)])
def test_quad_planes_full_apply(systems, monkeypatch, cfg, prec, term, tol):
    monkeypatch.setenv("WTD_QUAD_PLANES", "1")
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    say(f"quad planes: apply {prec} cfg={cfg} grid={s.n} term={term}")
    L = _ctx(s, nb, prec, TERMS[term])
    got = to_complex(L.apply(a))
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a, terms=TERMS[term]))
    say(f"  rel err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("cfg,prec,tol", [("p8", "fp64", 1e-10), ("p6", "fp64", 1e-10),
                                          ("p8", "fp32", 2e-5)])
def test_quad_planes_sampled_rows(systems, monkeypatch, cfg, prec, tol):
    """48^3 / Nocc = 140 (row-blocked exchange) and 96^3 (with the response
    term) on sampled rows."""
    monkeypatch.setenv("WTD_QUAD_PLANES", "1")
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    rows = [0, s.nocc // 2, s.nocc - 1]
    say(f"quad planes: apply {prec} cfg={cfg} grid={s.n} rows={rows}")
    L = _ctx(s, nb, prec)
    got = to_complex(L.apply(a))[:, rows]
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a, rows=rows))
    say(f"  rel err {err:.3e}")
    assert err <= tol


def test_quad_planes_davidson_and_backward(systems, monkeypatch):
    """FP64 Davidson on the 24^3 / Nocc = 128 system against the oracle's stored
    roots, and the backward against the oracle adjoint, on quad planes."""
    monkeypatch.setenv("WTD_QUAD_PLANES", "1")
    s = systems("p5")
    ref = json.load(open(os.path.join(GOLDEN, "roots_p5.json")))
    ev = np.array(ref["roots_hartree"])
    L = _ctx(s, s.cfg.nb, "fp64")
    omega, x, resid, it, st = L.davidson(s.cfg.nroots, s.cfg.nb, tol=1e-8, max_iter=100)
    err = np.max(np.abs(omega - ev[:s.cfg.nroots]) / np.abs(ev[:s.cfg.nroots]))
    say(f"quad planes: davidson fp64 p5: {it} iterations, max rel err {err:.3e}")
    assert st == 0 and err <= 1e-10
    a = trials_random(s, 2)
    g = trials_random(s, 2, offset=3000)
    ga, go = L.apply_bwd(a, g)
    ra, ro = oracle.grad_a(s, a, g), oracle.grad_occ(s, a, g)
    ea, eo = rel_err(to_complex(ga), ra), rel_err(to_complex(go)[None], ro[None])
    say(f"  backward: g_a rel err {ea:.3e}, g_occ rel err {eo:.3e}")
    L.close()
    assert ea <= 1e-10 and eo <= 1e-10
