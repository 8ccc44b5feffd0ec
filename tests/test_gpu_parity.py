"""GPU parity of the HIP fast path (through the C ABI) against the CPU oracle.

Tolerances: FP64 paths 1e-12 relative at n = 4 (the round-trip case) and a
looser FP64 bound at larger n, where the radix-2 recursion's intermediate skew
sub-transforms are ill conditioned (measured growth ~25x per doubling of n);
FP32 data paths 1e-5 relative.  Errors are max|y - y*| / max|y*|.
"""
import numpy as np
import pytest

import oracle
import paper_1807_10058_amd as fcc
import workloads
from oracle import fold_ref

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
RNG = np.random.default_rng(2024)
FP64_TOL = {1: 1e-14, 2: 1e-13, 4: 1e-12, 8: 1e-12, 16: 1e-11, 32: 1e-10, 64: 1e-8, 128: 1e-7}


def test_c1_n4_fp64_forward_inverse_roundtrip():
    n = 4
    x = workloads.uniform_fp64(n, 0)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP64)
    ref = oracle.forward(x, n)
    assert gu.maxrel(X, ref) <= 1e-12
    xi = gu.inverse(ref, n, fcc.FCC_PREC_FP64, real_out=True)
    assert gu.maxrel(xi, x) <= 1e-12
    xr = gu.inverse(X, n, fcc.FCC_PREC_FP64)
    assert gu.maxrel(xr, x) <= 1e-12
    assert gu.maxrel(xr, oracle.inverse(X, n)) <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 8, 16])
def test_fp64_complex_full(n):
    x = RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP64)
    ref = oracle.forward(x, n)
    assert gu.maxrel(X, ref) <= FP64_TOL[n]
    xi = gu.inverse(ref, n, fcc.FCC_PREC_FP64)
    assert gu.maxrel(xi, oracle.inverse(ref, n)) <= 10 * FP64_TOL[n]


@pytest.mark.parametrize("rst", [(0.31, 0.07, 0.23), (0.2, 0.45, 0.05)])
def test_fp64_generic_skew(rst):
    n = 8
    x = RNG.standard_normal(n ** 3)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP64, rst=rst)
    ref = oracle.forward(x, n, rst)
    assert gu.maxrel(X, ref) <= 1e-11
    xi = gu.inverse(ref, n, fcc.FCC_PREC_FP64, rst=rst, real_out=True)
    assert gu.maxrel(xi, x) <= 1e-10


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_fp32_full(n):
    x = RNG.uniform(-1, 1, n ** 3).astype(np.float32)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP32)
    ref = oracle.forward(x.astype(np.float64), n)
    assert gu.maxrel(X, ref) <= 1e-5


def test_fp32_n32_sampled_rows_and_fold():
    n = 32
    x = RNG.uniform(-1, 1, n ** 3).astype(np.float32)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP32)
    rows = gu.sample_rows(n, 128, 7)
    ref_rows = oracle.forward_rows(x.astype(np.float64), n, rows)
    assert gu.maxrel(X[rows], ref_rows) <= 1e-5
    assert gu.maxrel(X, fold_ref.fold_forward(x.astype(np.float64), n)) <= 1e-5


def test_c2_n64_gaussian_field_fp32():
    """n = 64 smooth field (16 Gaussians + N(0,0.01) noise), FP32 data."""
    n = 64
    x = workloads.gaussian_field(n, seed=1)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP32)
    rows = gu.sample_rows(n, 256, 101)
    ref_rows = oracle.forward_rows(x.astype(np.float64), n, rows)
    assert gu.maxrel(X[rows], ref_rows) <= 1e-5
    full = fold_ref.fold_forward(x.astype(np.float64), n)
    assert gu.maxrel(X, full) <= 1e-5


@pytest.mark.parametrize("n", [32, 64])
def test_fp32_roundtrip(n):
    x = RNG.standard_normal(n ** 3).astype(np.float32)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP32)
    xr = gu.inverse(X.astype(np.complex64), n, fcc.FCC_PREC_FP32, real_out=True)
    assert gu.maxrel(xr, x) <= 1e-5


@pytest.mark.parametrize("n", [16, 64])
def test_level0_fp32_option(n):
    """FCC_LEVEL0_FP32: the top level in FP32 arithmetic and storage, FP64
    below.  Rounding at the top level is not amplified by the recursion: the
    forward stays within the FP32 bound and the round trip within 1e-5."""
    x = RNG.standard_normal(n ** 3).astype(np.float32)
    X, _ = gu.forward(x, n, fcc.FCC_PREC_FP32, flags=fcc.FCC_LEVEL0_FP32)
    if n <= 16:
        ref = oracle.forward(x.astype(np.float64), n)
        assert gu.maxrel(X, ref) <= 1e-5
    else:
        rows = gu.sample_rows(n, 128, 5)
        assert gu.maxrel(X[rows], oracle.forward_rows(x.astype(np.float64), n, rows)) <= 1e-5
    xr = gu.inverse(X.astype(np.complex64), n, fcc.FCC_PREC_FP32, flags=fcc.FCC_LEVEL0_FP32, real_out=True)
    assert gu.maxrel(xr, x) <= 1e-5


def test_error_paths_on_gpu():
    import torch
    n = 4
    plan = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT)
    x = torch.zeros(n ** 3 + 4, dtype=torch.float32, device=gu.DEV)
    X = torch.zeros(n ** 3, dtype=torch.complex64, device=gu.DEV)
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_forward(plan, x.data_ptr() + 4, X)
    assert e.value.status == 1
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_forward(plan, X, X)
    assert e.value.status == 6


def test_batched_matches_single_calls():
    import torch
    ns = [2, 4, 8, 4]
    plans = [fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT) for n in ns]
    xs = [torch.from_numpy(RNG.standard_normal(n ** 3).astype(np.float32)).to(gu.DEV) for n in ns]
    outs = [torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV) for n in ns]
    fcc.fcc_dct_batched(plans, xs, outs, +1)
    torch.cuda.synchronize()
    for n, x, o in zip(ns, xs, outs):
        ref = oracle.forward(x.cpu().numpy().astype(np.float64), n)
        assert gu.maxrel(o.cpu().numpy(), ref) <= 1e-5
