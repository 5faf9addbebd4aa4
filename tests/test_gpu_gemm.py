"""The MFMA GEMM kernel against numpy (FP64 and FP32, both B layouts, ragged sizes)."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kmajor", [True, False])
@pytest.mark.parametrize("mnk", [(16, 16, 4), (32, 8, 950), (100, 12, 37), (39, 894, 9),
                                 (64, 64, 16), (130, 70, 33)])
def test_gemm(prec, kmajor, mnk):
    import torch
    from paper_2309_03513_amd import load_library
    lib = load_library()
    m, n, k = mnk
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(m * 1000 + n + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    Bst = B.T.copy() if kmajor else B.copy()
    dA = torch.tensor(A, dtype=dt, device="cuda")
    dB = torch.tensor(Bst, dtype=dt, device="cuda")
    dC = torch.zeros((m, n), dtype=dt, device="cuda")
    ldb = k if kmajor else n
    say(f"gemm {prec} kmajor={kmajor} m,n,k={mnk}")
    st = lib.wtd_debug_gemm(0 if prec == "fp64" else 1, m, n, k, ctypes.c_void_p(dA.data_ptr()),
                            k, ctypes.c_void_p(dB.data_ptr()), ldb, int(kmajor),
                            ctypes.c_void_p(dC.data_ptr()), n,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    C = dC.cpu().numpy().astype(np.float64)
    ref = A @ B
    err = np.abs(C - ref).max() / np.abs(ref).max()
    say(f"  max rel err {err:.3e}")
    if err > 1e-3:
        bad = np.argwhere(np.abs(C - ref) > 1e-3 * np.abs(ref).max())
        say(f"  first bad entries {bad[:8].tolist()}")
        i, j = bad[0]
        say(f"  C[{i},{j}]={C[i, j]} ref={ref[i, j]}; ref^T-match="
            f"{np.argwhere(np.abs(ref - C[i, j]) < 1e-9 * np.abs(ref).max())[:3].tolist()}")
    assert err <= (1e-13 if prec == "fp64" else 2e-6)
