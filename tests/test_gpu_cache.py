"""Pair-potential cache (wtd_cache_pairs): reusing tau between applies must give
the results of recomputing it, bit for bit, and every change of the occupied
orbitals (wtd_set_occ, the orbital gradient of the backward) must drop it."""
import numpy as np
import pytest
import torch

import oracle
from gen import trials_random
from paper_2309_03513_amd.wtd import WtdError
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu


def _ctx(s, nb, prec):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec)


def _same(x, y):
    return torch.equal(x, y)


@pytest.mark.parametrize("cfg,prec", [("c1", "fp64"), ("p5", "fp64"), ("p5", "fp32"), ("p1", "fp32")])
def test_cached_pairs_match_recomputed(systems, cfg, prec):
    s = systems(cfg)
    nb = s.cfg.nb
    a1 = trials_random(s, nb)
    a2 = trials_random(s, nb, offset=2007)
    say(f"pair cache cfg={cfg} prec={prec} nb={nb}")
    L = _ctx(s, nb, prec)
    r1 = L.apply(a1).clone()
    r2 = L.apply(a2).clone()
    L.cache_pairs(True)
    c1 = L.apply(a1).clone()      # forms and keeps the pairs
    c2 = L.apply(a2).clone()      # reuses them
    c1b = L.apply(a1).clone()
    torch.cuda.synchronize()
    assert _same(c1, r1) and _same(c2, r2) and _same(c1b, r1)
    # the cached result is still the operator: check against the oracle
    ref = oracle.apply_liouville(s, a2)
    err = rel_err(to_complex(c2), ref)
    say(f"  cached apply rel err {err:.3e}")
    assert err <= (1e-10 if prec == "fp64" else 2e-5)
    L.close()


def test_set_occ_drops_cached_pairs(systems):
    s = systems("p2")
    nb = s.cfg.nb
    a = trials_random(s, nb)
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(rng.standard_normal((s.nocc, s.nocc)))
    say("pair cache + set_occ p2")
    L = _ctx(s, nb, "fp64")
    L.cache_pairs(True)
    L.apply(a)
    L.set_occ(U.T @ s.c_occ)
    got = L.apply(a).clone()
    L.cache_pairs(False)
    ref = L.apply(a).clone()
    torch.cuda.synchronize()
    assert _same(got, ref)
    L.close()


def test_backward_drops_cached_pairs(systems):
    s = systems("c1")
    nb = s.cfg.nb
    a = trials_random(s, nb)
    g = trials_random(s, nb, offset=2003)
    say("pair cache + backward c1")
    L = _ctx(s, nb, "fp64")
    ref = L.apply(a).clone()
    L.cache_pairs(True)
    L.apply(a)
    L.apply_bwd(a, g)             # the orbital gradient reuses the pair buffer
    got = L.apply(a).clone()
    torch.cuda.synchronize()
    assert _same(got, ref)
    L.close()


def test_row_blocked_refuses_pair_cache(systems, monkeypatch):
    monkeypatch.setenv("WTD_ROW_BLOCK", "16")
    s = systems("p1")
    say("pair cache refused on the row-blocked path")
    L = _ctx(s, s.cfg.nb, "fp64")
    with pytest.raises(WtdError, match="WTD_ERR_SHAPE"):
        L.cache_pairs(True)
    L.cache_pairs(False)
    L.close()
