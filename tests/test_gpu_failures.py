"""Error paths forced from the host: non-finite inputs and a workspace cap.

Every case is rejected by the library before or after its kernels run; no
kernel is made to fault."""
import numpy as np
import pytest
import torch

import oracle
from gen import trials_random
from paper_2309_03513_amd import Liouville, WtdError
from paper_2309_03513_amd.wtd import set_workspace_limit
from tests.gpu_util import rel_err, say, to_complex

pytestmark = pytest.mark.gpu

NONFINITE, OOM = -6, -3


@pytest.mark.parametrize("what", ["c_occ", "c_cond", "fxc", "eps_occ"])
def test_create_rejects_nonfinite_system(systems, what):
    s = systems("c1")
    arr = np.array(getattr(s, what), copy=True)
    arr.flat[arr.size // 3] = np.nan if what != "fxc" else np.inf
    say(f"create with a non-finite {what} (expected WTD_ERR_NONFINITE)")
    with pytest.raises(WtdError) as e:
        Liouville(s.replace(**{what: arr}), max_nb=2, precision="fp64")
    assert e.value.status == NONFINITE
    assert what in str(e.value)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checked_apply_rejects_nan_trial(systems, prec):
    s = systems("c1")
    a = trials_random(s, 2)
    L = Liouville(s, max_nb=2, precision=prec)
    ref = L.apply(a).clone()
    L.set_checks(True)
    same = L.apply(a).clone()             # finite input: checks pass, same result
    torch.cuda.synchronize()
    assert torch.equal(same, ref)
    bad = a.copy()
    bad[1, 3, 7] = np.nan
    say(f"checked apply {prec} with a NaN trial coefficient (expected WTD_ERR_NONFINITE)")
    with pytest.raises(WtdError) as e:
        L.apply(bad)
    assert e.value.status == NONFINITE and "trial block" in str(e.value)
    with pytest.raises(WtdError) as e:
        L.apply_bwd(a, bad)
    assert e.value.status == NONFINITE and "cotangent" in str(e.value)
    L.set_checks(False)
    after = L.apply(a).clone()            # the context is still usable
    L.close()
    torch.cuda.synchronize()
    assert torch.equal(after, ref)
    err = rel_err(to_complex(ref), oracle.apply_liouville(s, a))
    assert err <= (1e-10 if prec == "fp64" else 2e-5)


def test_workspace_limit_refuses_large_context(systems):
    s = systems("p1")
    L = Liouville(s, max_nb=5, precision="fp64")
    need = L.workspace_bytes()
    L.close()
    say(f"workspace cap below the {need} bytes a p1 context needs (expected WTD_ERR_OOM)")
    try:
        set_workspace_limit(need // 2)
        with pytest.raises(WtdError) as e:
            Liouville(s, max_nb=5, precision="fp64")
        assert e.value.status == OOM and "limit" in str(e.value)
        set_workspace_limit(need + (1 << 20))
        L = Liouville(s, max_nb=5, precision="fp64")   # fits under a cap above its size
        a = trials_random(s, 5)
        err = rel_err(to_complex(L.apply(a)), oracle.apply_liouville(s, a))
        L.close()
        assert err <= 1e-10
    finally:
        set_workspace_limit(0)
