"""Row-blocked exchange (the path for Nocc > 128) against the FP64 oracle.

Above 128 occupied orbitals the pair triangle is processed in blocks of 64
rows, so only one block pair of pair potentials is held at a time.  The same
path can be forced for small systems (WTD_ROW_BLOCK = 16 / 32 / 48), which
gives ragged last blocks, single-block systems and several block pairs at
sizes the oracle finishes in seconds.  The spin-flip operator (c_K = 0: D and
the exchange term only) is checked on the same path."""
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


@pytest.mark.parametrize("cfg,rb", [("c1", 16), ("p1", 16), ("p2", 16), ("p3", 16), ("p3", 32),
                                    ("p3", 48)])
def test_forced_blocks_fp64(systems, monkeypatch, cfg, rb):
    monkeypatch.setenv("WTD_ROW_BLOCK", str(rb))
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    for term in ("K1D", "ALL"):
        say(f"blocked apply fp64 cfg={cfg} row_block={rb} term={term} nb={nb}")
        L = _ctx(s, nb, "fp64", TERMS[term])
        got = to_complex(L.apply(a))
        L.close()
        err = rel_err(got, oracle.apply_liouville(s, a, terms=TERMS[term]))
        say(f"  rel err {err:.3e}")
        assert err <= 1e-10


def test_forced_blocks_fp32(systems, monkeypatch):
    monkeypatch.setenv("WTD_ROW_BLOCK", "16")
    s = systems("p1")
    a, _ = trials_in_span(s, s.cfg.nb)
    say("blocked apply fp32 p1 row_block=16")
    L = _ctx(s, s.cfg.nb, "fp32")
    got = to_complex(L.apply(a))
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a))
    say(f"  rel err {err:.3e}")
    assert err <= 2e-5


@pytest.mark.parametrize("rb,nb", [("16", 16), ("48", 16), ("64", 32), ("32", 48), ("48", 11)])
def test_forced_blocks_fp32_interleaved(systems, monkeypatch, rb, nb):
    """FP32 row-blocked exchange: interleaved pair potentials and the
    register-operand block contraction (32 trials per pass; Nb = 48 takes a
    second, half-empty pass, Nb = 11 one pass with 21 empty trials), blocks of
    16 to 64 rows with a ragged last block (128 = 48 + 48 + 32), compared
    element by element with the oracle."""
    monkeypatch.setenv("WTD_ROW_BLOCK", rb)
    s = systems("p5")
    a = trials_random(s, nb)
    say(f"blocked apply fp32 p5 row_block={rb} nb={nb}")
    L = _ctx(s, nb, "fp32")
    got = to_complex(L.apply(a))
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a))
    say(f"  rel err {err:.3e}")
    assert err <= 2e-5


@pytest.mark.parametrize("term", ["K1D", "ALL"])
def test_nocc_144_fp64(systems, term):
    """Nocc = 144 takes the blocked path by itself (blocks of 64, 64, 16 rows)."""
    s = systems("p4")
    a = trials_random(s, 2)
    say(f"nocc=144 apply fp64 term={term}")
    L = _ctx(s, 2, "fp64", TERMS[term])
    got = to_complex(L.apply(a))
    L.close()
    err = rel_err(got, oracle.apply_liouville(s, a, terms=TERMS[term]))
    say(f"  rel err {err:.3e}")
    assert err <= 1e-10


def test_nocc_144_fp32_and_spin_flip(systems):
    s = systems("p4")
    a, _ = trials_in_span(s, 2)
    say("nocc=144 apply fp32")
    L = _ctx(s, 2, "fp32")
    got = to_complex(L.apply(a))
    L.close()
    assert rel_err(got, oracle.apply_liouville(s, a)) <= 2e-5
    sf = s.replace(c_k=0.0)
    say("nocc=144 spin-flip (c_K = 0) fp64")
    L = _ctx(sf, 2)
    got = to_complex(L.apply(a))
    L.close()
    assert rel_err(got, oracle.apply_liouville(sf, a)) <= 1e-10


@pytest.mark.parametrize("cfg,rb,terms", [("p1", 16, 7), ("p3", 16, 4), ("p2", 16, 7)])
def test_forced_blocks_backward(systems, monkeypatch, cfg, rb, terms):
    monkeypatch.setenv("WTD_ROW_BLOCK", str(rb))
    s = systems(cfg)
    nb = min(s.cfg.nb, 3)
    a = trials_random(s, nb)
    g = trials_random(s, nb, offset=3000)
    say(f"blocked backward fp64 cfg={cfg} row_block={rb} terms={terms}")
    L = _ctx(s, nb, "fp64", terms)
    ga, go = L.apply_bwd(a, g)
    L.close()
    ea = rel_err(to_complex(ga), oracle.grad_a(s, a, g, terms=terms))
    eo = rel_err(to_complex(go)[None], oracle.grad_occ(s, a, g, terms=terms)[None])
    say(f"  rel err g_a {ea:.3e}, g_occ {eo:.3e}")
    assert ea <= 1e-10 and eo <= 1e-10


def test_blocked_davidson_spin_flip_matches_dense(systems, monkeypatch):
    """Spin-flip spectrum (c_K = 0) from the GPU Davidson on the blocked path
    against the dense oracle matrix of the same operator."""
    monkeypatch.setenv("WTD_ROW_BLOCK", "16")
    s = systems("p1").replace(c_k=0.0)
    n = s.nocc * s.ncond
    M = oracle.apply_transition(s, np.eye(n).reshape(n, s.nocc, s.ncond)).reshape(n, n)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    say("blocked davidson fp64 p1 spin-flip")
    L = _ctx(s, 4)
    omega, x, resid, nit, st = L.davidson(4, 4, tol=1e-8, max_iter=200)
    L.close()
    say(f"  omega={omega} iters={nit} status={st}")
    assert st == 0
    assert np.max(np.abs(omega - ev[:4]) / np.abs(ev[:4])) <= 1e-10
