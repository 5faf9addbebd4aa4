"""Autotuner (wtd_autotune): the chosen launch shape is one of the candidates
and the tuned context still computes the operator (oracle parity); the pair
potentials, and so the K1d-only result, do not depend on the pair batch."""
import pytest
import torch

import oracle
from gen import trials_random
from paper_2309_03513_amd.wtd import WtdError
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu


def _ctx(s, nb, prec, terms=7):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec, terms=terms)


@pytest.mark.parametrize("cfg,prec,tol", [("c1", "fp64", 1e-10), ("p5", "fp64", 1e-10),
                                          ("p5", "fp32", 2e-5), ("p1", "fp32", 2e-5)])
def test_autotuned_apply_matches_oracle(systems, cfg, prec, tol):
    s = systems(cfg)
    nb = s.cfg.nb
    a = trials_random(s, nb)
    L = _ctx(s, nb, prec)
    chunk, groups = L.autotune(nb, reps=2)
    say(f"autotune cfg={cfg} prec={prec}: pair batch {chunk}, density split {groups}")
    npack = (s.nocc * (s.nocc + 1) // 2 + 1) // 2
    assert groups in (1, 2, 4, 8)
    assert 1 <= chunk <= min(512, npack)
    err = rel_err(to_complex(L.apply(a)), oracle.apply_liouville(s, a))
    say(f"  rel err after tuning {err:.3e}")
    assert err <= tol
    L.close()


def test_pair_batch_does_not_change_k1d(systems, monkeypatch):
    """K1d alone (no density response) is bitwise the same for any pair batch."""
    s = systems("p1")
    nb = s.cfg.nb
    a = trials_random(s, nb)
    outs = []
    for chunk in ("16", "40", "512"):
        monkeypatch.setenv("WTD_PAIR_CHUNK", chunk)
        L = _ctx(s, nb, "fp64", terms=4)
        outs.append(L.apply(a).clone())
        L.close()
    torch.cuda.synchronize()
    say("K1d with pair batches 16, 40, 512")
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_autotune_rejects_bad_arguments(systems):
    s = systems("c1")
    L = _ctx(s, s.cfg.nb, "fp64")
    with pytest.raises(WtdError, match="WTD_ERR_SHAPE"):
        L.autotune(s.cfg.nb + 1)
    with pytest.raises(WtdError, match="WTD_ERR_ARG"):
        L.autotune(1, reps=0)
    L.close()
