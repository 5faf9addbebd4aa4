"""Pins of the oracle adjoint against finite differences of the oracle forward.

E = Re sum conj(g) (L a) is linear in a and exactly quadratic in the occupied
coefficients (D and the projector do not depend on them), so central
differences are exact up to rounding; h = 1e-4 in FP64.
"""
import numpy as np
import pytest

import oracle
from gen import trials_random

H = 1e-4


def _dirs(s, nb, seed):
    rng = np.random.default_rng(seed)
    def rnd(shape):
        x = rng.standard_normal(shape + (2,))
        return x[..., 0] + 1j * x[..., 1]
    return rnd((nb, s.nocc, s.npw)), rnd((s.nocc, s.npw))


@pytest.mark.parametrize("terms", [7, 2, 4, 1])
def test_grad_a_matches_central_difference(systems, terms):
    s = systems("p2")
    a = trials_random(s, 2)
    g = trials_random(s, 2, offset=3000)
    da, _ = _dirs(s, 2, 5)
    ga = oracle.grad_a(s, a, g, terms=terms)
    fd = (oracle.energy(s, a + H * da, g, terms) - oracle.energy(s, a - H * da, g, terms)) / (2 * H)
    an = np.sum(ga.real * da.real + ga.imag * da.imag)
    assert abs(an - fd) <= 1e-9 * max(abs(fd), 1e-12)


@pytest.mark.parametrize("terms", [7, 2, 4])
def test_grad_occ_matches_central_difference(systems, terms):
    s = systems("p2")
    a = trials_random(s, 2)
    g = trials_random(s, 2, offset=3000)
    _, dc = _dirs(s, 2, 6)
    go = oracle.grad_occ(s, a, g, terms=terms)
    ep = oracle.energy(s, a, g, terms, occ=s.c_occ + H * dc)
    em = oracle.energy(s, a, g, terms, occ=s.c_occ - H * dc)
    fd = (ep - em) / (2 * H)
    an = np.sum(go.real * dc.real + go.imag * dc.imag)
    assert abs(an - fd) <= 1e-9 * max(abs(fd), 1e-12), (an, fd)


def test_grad_occ_is_zero_for_d_only(systems):
    s = systems("c1")
    a = trials_random(s, 1)
    g = trials_random(s, 1, offset=3000)
    assert np.abs(oracle.grad_occ(s, a, g, terms=1)).max() == 0.0


def test_grad_a_dot_product_identity(systems):
    """<g_a(g), d> = <g, L d> for any d (the transpose property)."""
    s = systems("c1")
    g = trials_random(s, 2, offset=3000)
    d = trials_random(s, 2, offset=4000)
    ga = oracle.grad_a(s, None, g)
    ld = oracle.apply_liouville(s, d)
    lhs = np.sum(ga.real * d.real + ga.imag * d.imag)
    rhs = np.sum(g.real * ld.real + g.imag * ld.imag)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
