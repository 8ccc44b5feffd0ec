"""The allocation-free forward entry point (scratch in the library's static
device array) gives the same result bits as fcc_dct_forward, on two calls in a
row with the second smaller, and both match the oracle within the FP32 1e-5
relative bound (Sec. IV-A, Def. 2).  Calls go through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1807_10058_amd as fcc

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _static_forward(plan, x, X):
    lib = ctypes.CDLL(fcc.lib_path())
    lib.fcc_dct_forward_static.argtypes = [ctypes.c_void_p] * 4
    lib.fcc_dct_forward_static.restype = ctypes.c_int
    return lib.fcc_dct_forward_static(plan.handle, x.data_ptr(), X.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)


def _case(n, seed, prec=fcc.FCC_PREC_FP32):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, n ** 3)
    real = torch.float64 if prec == fcc.FCC_PREC_FP64 else torch.float32
    cplx = torch.complex128 if prec == fcc.FCC_PREC_FP64 else torch.complex64
    plan = fcc.fcc_dct_plan(n, prec=prec, flags=fcc.FCC_REAL_INPUT)
    xt = torch.from_numpy(x).to(DEV, real)
    ref_t = torch.empty(n ** 3, dtype=cplx, device=DEV)
    got_t = torch.full((n ** 3,), float("nan"), dtype=cplx, device=DEV)
    fcc.fcc_dct_forward(plan, xt, ref_t)
    assert _static_forward(plan, xt, got_t) == 0
    torch.cuda.synchronize()
    return x.astype(np.float32 if prec != fcc.FCC_PREC_FP64 else np.float64), ref_t.cpu().numpy(), got_t.cpu().numpy()


@pytest.mark.parametrize("sizes", [(64, 16), (32, 8)])
def test_static_forward_matches_forward_twice(sizes):
    for k, n in enumerate(sizes):
        x, ref, got = _case(n, 100 + k)
        assert np.array_equal(ref, got), n
        rows = np.random.default_rng(7 + k).choice(n ** 3, 24, replace=False)
        want = oracle.forward_rows(x.astype(np.float64), n, rows)
        assert np.abs(got[rows] - want).max() / np.abs(want).max() <= 1e-5


def test_static_forward_fp64_and_dense():
    x, ref, got = _case(16, 5, fcc.FCC_PREC_FP64)
    assert np.array_equal(ref, got)
    x, ref, got = _case(8, 6, fcc.FCC_PREC_SPLIT_BF16)
    assert np.array_equal(ref, got)


def test_static_forward_rejects_sizes_above_the_array():
    plan = fcc.fcc_dct_plan(128, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT)
    x = torch.zeros(128 ** 3, dtype=torch.float32, device=DEV)
    X = torch.empty(128 ** 3, dtype=torch.complex64, device=DEV)
    assert _static_forward(plan, x, X) == 6  # FCC_ERR_UNSUPPORTED
