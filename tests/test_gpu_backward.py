"""The HIP backward apply against the oracle adjoint and finite differences."""
import numpy as np
import pytest

import oracle
from gen import trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu


def _ctx(s, nb, prec="fp64", terms=7):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec, terms=terms)


@pytest.mark.parametrize("cfg,terms", [("c1", 7), ("p2", 7), ("p2", 2), ("p2", 4), ("p1", 7),
                                       ("p3", 7)])
def test_backward_fp64_matches_oracle_adjoint(systems, cfg, terms):
    s = systems(cfg)
    nb = min(s.cfg.nb, 3)
    a = trials_random(s, nb)
    g = trials_random(s, nb, offset=3000)
    say(f"backward fp64 cfg={cfg} terms={terms} nb={nb}")
    L = _ctx(s, nb, "fp64", terms)
    ga, go = L.apply_bwd(a, g)
    L.close()
    ga, go = to_complex(ga), to_complex(go)
    ra = oracle.grad_a(s, a, g, terms=terms)
    ro = oracle.grad_occ(s, a, g, terms=terms)
    ea, eo = rel_err(ga, ra), rel_err(go[None], ro[None])
    say(f"  rel err g_a {ea:.3e}, g_occ {eo:.3e}")
    assert ea <= 1e-10 and eo <= 1e-10


def test_backward_fp32(systems):
    s = systems("p1")
    a = trials_random(s, 3)
    g = trials_random(s, 3, offset=3000)
    say("backward fp32 p1")
    L = _ctx(s, 3, "fp32")
    ga, go = L.apply_bwd(a, g)
    L.close()
    ea = rel_err(to_complex(ga), oracle.grad_a(s, a, g))
    eo = rel_err(to_complex(go)[None], oracle.grad_occ(s, a, g)[None])
    say(f"  rel err g_a {ea:.3e}, g_occ {eo:.3e}")
    assert ea <= 1e-4 and eo <= 1e-4


def test_backward_occ_matches_gpu_central_difference(systems):
    """E is exactly quadratic in the occupied coefficients: central differences
    of the GPU forward (h = 1e-4, FP64) equal <g_occ, d> up to rounding."""
    s = systems("c1")
    a = trials_random(s, 2)
    g = trials_random(s, 2, offset=3000)
    rng = np.random.default_rng(11)
    d = rng.standard_normal((s.nocc, s.npw)) + 1j * rng.standard_normal((s.nocc, s.npw))
    h = 1e-4
    say("backward fp64 vs GPU central difference, c1")
    L = _ctx(s, 2)
    _, go = L.apply_bwd(a, g)
    go = to_complex(go)

    def energy(c):
        L.set_occ(c)
        la = to_complex(L.apply(a))
        return float(np.sum(g.real * la.real + g.imag * la.imag))

    fd = (energy(s.c_occ + h * d) - energy(s.c_occ - h * d)) / (2 * h)
    L.close()
    an = float(np.sum(go.real * d.real + go.imag * d.imag))
    say(f"  analytic {an:.12e} fd {fd:.12e}")
    assert abs(an - fd) <= 1e-8 * abs(fd)


def test_autograd_function_matches_oracle(systems):
    import torch
    from paper_2309_03513_amd import Liouville
    from paper_2309_03513_amd.autograd import liouville_apply
    s = systems("p2")
    a_np = trials_random(s, 2)
    g_np = trials_random(s, 2, offset=3000)
    say("autograd LiouvilleApply fp64 p2")
    op = Liouville(s, max_nb=2, precision="fp64")
    to_t = lambda x: torch.tensor(np.stack([x.real, x.imag], -1), dtype=torch.float64,
                                  device="cuda", requires_grad=True)
    a, c = to_t(a_np), to_t(s.c_occ)
    gt = torch.tensor(np.stack([g_np.real, g_np.imag], -1), dtype=torch.float64, device="cuda")
    la = liouville_apply(a, c, op)
    (la * gt).sum().backward()
    op.close()
    assert rel_err(to_complex(a.grad), oracle.grad_a(s, a_np, g_np)) <= 1e-10
    assert rel_err(to_complex(c.grad)[None], oracle.grad_occ(s, a_np, g_np)[None]) <= 1e-10
