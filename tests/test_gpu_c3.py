"""The 108^3 / Nocc = 432 workload (215-atom-cell size) on the row-blocked path.

The oracle cannot apply the whole operator at this size in test time, so the
GPU apply is checked on sampled output rows: the oracle computes R_v for a few
occupied indices v (with the exchange sum over every v') and the full
projection, for the spin-conserving operator (c_K = 2) and the spin-flip one
(c_K = 0, exchange only).  The oracle work takes minutes of host time, so
these run with WTD_SLOW_TESTS=1."""
import os

import numpy as np
import pytest

import oracle
from gen import trials_random
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu

ROWS = [0, 215, 431]


@pytest.fixture(scope="module")
def c3_case(systems):
    import oracle.planewave as pw
    pw._WORKERS = len(os.sched_getaffinity(0))
    s = systems("c3")
    a = trials_random(s, 2)
    say("oracle rows at 108^3 / Nocc = 432: exchange + D")
    ref_d_k1d = oracle.apply_liouville(s, a, terms=oracle.TERM_D | oracle.TERM_K1D, rows=ROWS,
                                       progress=say)
    say("oracle rows at 108^3 / Nocc = 432: response term")
    ref_k1e = oracle.apply_liouville(s, a, terms=oracle.TERM_K1E, rows=ROWS, progress=say)
    return s, a, ref_d_k1d, ref_k1e


def _apply(s, a, prec):
    from paper_2309_03513_amd import Liouville
    L = Liouville(s, max_nb=a.shape[0], precision=prec)
    out = to_complex(L.apply(a))
    L.close()
    return out


@pytest.mark.slow
def test_c3_spin_conserving_rows_fp32(c3_case):
    s, a, ref_d_k1d, ref_k1e = c3_case
    say("c3 spin-conserving apply fp32")
    got = _apply(s, a, "fp32")[:, ROWS]
    err = rel_err(got, ref_d_k1d + ref_k1e)
    say(f"  rows {ROWS} rel err {err:.3e}")
    assert err <= 2e-5


def test_c3_fp64_plane_does_not_fit_lds(systems):
    """A 108 x 108 FP64 plane (187 KB) exceeds the 160 KB of LDS of one
    workgroup: context creation reports WTD_ERR_SHAPE instead of launching."""
    from paper_2309_03513_amd import Liouville, WtdError
    s = systems("c3")
    say("c3 fp64 context creation (expected shape error)")
    with pytest.raises(WtdError) as e:
        Liouville(s, max_nb=1, precision="fp64")
    assert e.value.status == -2


@pytest.mark.slow
def test_c3_spin_flip_rows_fp32(c3_case):
    s, a, ref_d_k1d, _ = c3_case
    say("c3 spin-flip apply fp32 (c_K = 0)")
    got = _apply(s.replace(c_k=0.0), a, "fp32")[:, ROWS]
    err = rel_err(got, ref_d_k1d)
    say(f"  rows {ROWS} rel err {err:.3e}")
    assert err <= 2e-5
