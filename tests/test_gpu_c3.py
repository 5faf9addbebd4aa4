"""The 108^3 / Nocc = 432 workload (215-atom-cell size) on the row-blocked path.

The oracle cannot apply the whole operator at this size in test time, so the
GPU apply is checked on sampled output rows that the oracle wrote once:
tests/golden/rows_c3.npz holds, for the seeded two-trial block of
gen.trials_random, the rows v = 0, 215, 431 of the D, K1d and K1e terms
separately (written by tests/golden/make_golden.py c3rows, which calls only the
oracle and the generator; the exchange sum runs over every v').  Each term is
checked on its own (the D term dominates the sum, so a K-term mistake could
hide under it), in FP32 and in FP64, then the spin-conserving operator
(c_K = 2) and the spin-flip one (c_K = 0, exchange only)."""
import os

import numpy as np
import pytest

import oracle
from gen import trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rows_c3.npz")


@pytest.fixture(scope="module")
def c3_case(systems):
    ref = np.load(GOLDEN)
    s = systems("c3")
    a = trials_random(s, int(ref["nb"]))
    return s, a, [int(v) for v in ref["rows"]], {k: ref[k] for k in ("d", "k1d", "k1e")}


def _apply(s, a, rows, prec, terms=oracle.TERM_ALL):
    from paper_2309_03513_amd import Liouville
    L = Liouville(s, max_nb=a.shape[0], precision=prec, terms=terms)
    out = to_complex(L.apply(a))[:, rows]
    L.close()
    return out


@pytest.mark.parametrize("term", ["k1d", "k1e", "d"])
def test_c3_term_rows_fp32(c3_case, term):
    s, a, rows, ref = c3_case
    mask = {"d": oracle.TERM_D, "k1d": oracle.TERM_K1D, "k1e": oracle.TERM_K1E}[term]
    say(f"c3 {term} rows {rows} fp32")
    err = rel_err(_apply(s, a, rows, "fp32", mask), ref[term])
    say(f"  rel err {err:.3e}")
    assert err <= 2e-5


def test_c3_spin_conserving_rows_fp32(c3_case):
    s, a, rows, ref = c3_case
    say("c3 spin-conserving apply fp32")
    err = rel_err(_apply(s, a, rows, "fp32"), ref["d"] + ref["k1d"] + ref["k1e"])
    say(f"  rows {rows} rel err {err:.3e}")
    assert err <= 2e-5


def test_c3_spin_flip_rows_fp32(c3_case):
    s, a, rows, ref = c3_case
    say("c3 spin-flip apply fp32 (c_K = 0)")
    err = rel_err(_apply(s.replace(c_k=0.0), a, rows, "fp32"), ref["d"] + ref["k1d"])
    say(f"  rows {rows} rel err {err:.3e}")
    assert err <= 2e-5


@pytest.mark.parametrize("term", ["k1d", "k1e", "d"])
def test_c3_term_rows_fp64(c3_case, term):
    """FP64 at 108^3: the 108 x 108 FP64 plane (187 KB) does not fit in LDS, so
    the plane transforms run on the register-quad kernels (lines in registers,
    one LDS transpose per 2D FFT)."""
    s, a, rows, ref = c3_case
    mask = {"d": oracle.TERM_D, "k1d": oracle.TERM_K1D, "k1e": oracle.TERM_K1E}[term]
    say(f"c3 {term} rows {rows} fp64")
    err = rel_err(_apply(s, a, rows, "fp64", mask), ref[term])
    say(f"  rel err {err:.3e}")
    assert err <= 1e-10
