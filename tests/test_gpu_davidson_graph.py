"""Davidson with every step after the first replayed from a HIP graph (a
context on its own stream) gives the eigenpairs of the eager run bit for bit,
for the all-pairs, single-block and row-blocked exchange, and its roots match
the dense eigenvalues of the oracle's operator."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _dense_roots(s, k):
    n = s.nocc * s.ncond
    M = oracle.apply_transition(s, np.eye(n).reshape(n, s.nocc, s.ncond)).reshape(n, n)
    return np.linalg.eigvalsh(0.5 * (M + M.T))[:k]


@pytest.mark.parametrize("cfg,prec,rb", [("c1", "fp64", None), ("p1", "fp32", None),
                                         ("p1", "fp64", "16")])
def test_davidson_graphs_match_eager(systems, monkeypatch, cfg, prec, rb):
    from paper_2309_03513_amd import Liouville
    if rb is not None:
        monkeypatch.setenv("WTD_ROW_BLOCK", rb)
    s = systems(cfg)
    nb = s.cfg.nb
    res = {}
    for graphs in ("0", "1"):
        monkeypatch.setenv("WTD_DAVIDSON_GRAPHS", graphs)
        st = torch.cuda.Stream()
        L = Liouville(s, max_nb=nb, precision=prec, stream=st)
        om, x, r, it, status = L.davidson(s.cfg.nroots, nb, tol=1e-8 if prec == "fp64" else 1e-5,
                                          max_iter=100)
        torch.cuda.synchronize()
        res[graphs] = (om.copy(), x.clone(), it)
        L.close()
    say(f"davidson {cfg} {prec} rb={rb}: {res['1'][2]} iterations, graphs vs eager")
    assert res["0"][2] == res["1"][2]
    assert np.array_equal(res["0"][0], res["1"][0])
    assert torch.equal(res["0"][1], res["1"][1])
    ev = _dense_roots(s, s.cfg.nroots)
    err = np.abs(res["1"][0] - ev)
    say(f"  vs the oracle's dense eigenvalues: max |d omega| {err.max():.3e} Ha")
    if prec == "fp64":
        assert np.max(err / np.abs(ev)) <= 1e-10
    else:
        assert err.max() <= 3.674932e-5
