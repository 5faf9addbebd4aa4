"""wtd_davidson_noalloc (the Davidson run in the library's static device array)
against wtd_davidson on the same contexts, through the C ABI: two runs in a
row, the second on a smaller system, then the first system again (the array
keeps the previous run's contents, which must not matter), and a run that does
not fit in the array."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _same_run(ref, got, rtol):
    om_r, x_r, rn_r, it_r, st_r = ref
    om_g, x_g, rn_g, it_g, st_g = got
    assert st_g == st_r and it_g == it_r, (st_r, it_r, st_g, it_g)
    err = float(np.max(np.abs(om_g - om_r) / np.abs(om_r)))
    xr = x_r.cpu().numpy()
    xg = x_g.cpu().numpy()
    xerr = 0.0
    for k in range(xr.shape[0]):
        sgn = 1.0 if np.sum(xr[k] * xg[k]) >= 0 else -1.0
        xerr = max(xerr, float(np.max(np.abs(xg[k] - sgn * xr[k])) / np.max(np.abs(xr[k]))))
    say(f"  omega rel err {err:.2e}, x elementwise {xerr:.2e}, iterations {it_g}")
    assert err <= rtol
    assert xerr <= 1e3 * rtol
    assert np.all(np.abs(rn_g - rn_r) <= 1e3 * rtol * np.maximum(np.abs(rn_r), 1e-12))


def test_davidson_noalloc_matches_davidson(systems):
    from paper_2309_03513_amd import Liouville
    big = systems("p5")     # 24^3, Nocc = 128, Nc = 16: the all-pairs FP32 contraction
    small = systems("c1")   # 24^3, Nocc = Nc = 8
    say("noalloc Davidson, first run: 24^3 / Nocc = 128 / Nc = 16, FP32 bulk, 4 roots, nb = 8")
    L = Liouville(big, max_nb=8, precision="fp32")
    ref = L.davidson(4, 8, tol=1e-5, max_iter=60)
    got1 = L.davidson_noalloc(4, 8, tol=1e-5, max_iter=60)
    _same_run(ref, got1, 1e-10)

    say("noalloc Davidson, second run, smaller system: 24^3 / Nocc = Nc = 8, FP64, 4 roots, nb = 4")
    S = Liouville(small, max_nb=4, precision="fp64")
    ref_s = S.davidson(4, 4, tol=1e-8, max_iter=60)
    got_s = S.davidson_noalloc(4, 4, tol=1e-8, max_iter=60)
    _same_run(ref_s, got_s, 1e-10)
    S.close()

    say("noalloc Davidson, the first system again (array holds the small run's contents)")
    got2 = L.davidson_noalloc(4, 8, tol=1e-5, max_iter=60)
    _same_run(got1, got2, 0.0)
    L.close()


def test_davidson_noalloc_rejects_oversized_run(systems):
    """A basis of 256 vectors over the 16,384 transitions of the 72^3 / Nocc = 128
    system needs 2 x 32 MiB for the basis and its products alone."""
    from paper_2309_03513_amd import Liouville, WtdError
    c2 = systems("c2")
    say("noalloc Davidson beyond the static array: 72^3 / Nocc = Nc = 128, nb = 1, max_sub = 256")
    L = Liouville(c2, max_nb=1, precision="fp32")
    with pytest.raises(WtdError) as e:
        L.davidson_noalloc(1, 1, tol=1e-5, max_iter=2, max_sub=256)
    L.close()
    say(f"  {e.value}")
    assert e.value.status == -2
    assert "bytes of scratch" in str(e.value)
