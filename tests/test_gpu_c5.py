"""The backward apply at the benchmark size: 72^3 grid, Nocc = 128, 16 trials.

The oracle's adjoint at this size costs minutes of host time, so the full-size
checks use properties that hold exactly at any size (the oracle adjoint itself
is compared element by element on smaller systems in test_gpu_backward.py):
* E = Re sum conj(g) (L a) is exactly quadratic in the occupied coefficients,
  so a central difference of two FP64 forward applies (h = 1e-4) equals
  <g_occ, d> up to rounding;
* E is linear in a, so <g_a, d_a> equals E(a + d_a) - E(a) = <g, L d_a>;
* the FP32 backward agrees with the FP64 one to FP32 accuracy."""
import numpy as np
import pytest

from gen import trials_in_span, trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu


def _ctx(s, nb, prec):
    from paper_2309_03513_amd import Liouville
    return Liouville(s, max_nb=nb, precision=prec)


def _dot(x, y):
    return float(np.sum(x.real * y.real + x.imag * y.imag))


@pytest.fixture(scope="module")
def c5(systems):
    s = systems("c2")
    a, _ = trials_in_span(s, 16)
    g = trials_random(s, 16, offset=3000)
    rng = np.random.default_rng(s.cfg.seed + 2000)
    env = np.exp(-np.sum((np.asarray(s.mill) * (2 * np.pi / s.cell)) ** 2, axis=1) / 4)
    d_occ = (rng.standard_normal((s.nocc, s.npw)) + 1j * rng.standard_normal((s.nocc, s.npw))) * env
    d_occ[:, 0] = d_occ[:, 0].real
    d_a = trials_random(s, 16, offset=4000)
    say("backward fp64 at 72^3 / Nocc = 128 / Nb = 16")
    L = _ctx(s, 16, "fp64")
    ga, go = L.apply_bwd(a, g)
    ga, go = to_complex(ga), to_complex(go)
    yield s, a, g, d_occ, d_a, L, ga, go
    L.close()


def test_c5_occ_gradient_vs_central_difference(c5):
    s, a, g, d_occ, _, L, _, go = c5
    h = 1e-4

    def energy(c):
        L.set_occ(c)
        return _dot(g, to_complex(L.apply(a)))

    say("central difference of two fp64 applies, h = 1e-4")
    fd = (energy(s.c_occ + h * d_occ) - energy(s.c_occ - h * d_occ)) / (2 * h)
    L.set_occ(s.c_occ)
    an = _dot(go, d_occ)
    say(f"  analytic {an:.12e} fd {fd:.12e}")
    assert abs(an - fd) <= 1e-8 * abs(fd)


def test_c5_trial_gradient_dot_product(c5):
    _, _, g, _, d_a, L, ga, _ = c5
    say("dot-product test <g_a, d_a> = <g, L d_a>")
    lhs = _dot(ga, d_a)
    rhs = _dot(g, to_complex(L.apply(d_a)))
    say(f"  {lhs:.12e} vs {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_c5_fp32_backward_vs_fp64(c5):
    s, a, g, _, _, _, ga, go = c5
    say("backward fp32 at 72^3 / Nocc = 128 / Nb = 16")
    L32 = _ctx(s, 16, "fp32")
    ga32, go32 = L32.apply_bwd(a, g)
    L32.close()
    ea = rel_err(to_complex(ga32), ga)
    eo = rel_err(to_complex(go32)[None], go[None])
    say(f"  rel err vs fp64: g_a {ea:.3e}, g_occ {eo:.3e}")
    assert ea <= 1e-4 and eo <= 1e-4

