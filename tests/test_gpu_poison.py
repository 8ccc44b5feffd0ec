"""Scratch poisoning (FCC_POISON_SCRATCH=1): every scratch buffer a plan or a
batched call allocates starts as all-ones bytes (NaN in FP32 and FP64).  The
results must equal, bit for bit, those of plans with ordinary scratch: no
kernel reads scratch it has not written."""
import os

import numpy as np
import pytest
import torch

import paper_1807_10058_amd as fcc

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
RNG = np.random.default_rng(99)

CASES = [
    (16, fcc.FCC_PREC_FP64, 0),
    (32, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT),
    (64, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_BASE),
    (64, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_LEVEL0_FP32),
    (32, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_FFT),
    (16, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_HERMITIAN_PACKED),
    (16, fcc.FCC_PREC_FP64, fcc.FCC_TRANSPOSED),
    (8, fcc.FCC_PREC_SPLIT_BF16, fcc.FCC_REAL_INPUT),
]


def _round_trip(n, prec, flags, x):
    plan = fcc.fcc_dct_plan(n, prec=prec, flags=flags)
    cd = torch.complex128 if prec == fcc.FCC_PREC_FP64 else torch.complex64
    X = torch.empty(fcc.fcc_dct_packed_size(plan), dtype=cd, device=gu.DEV)
    y = torch.empty_like(x)
    fcc.fcc_dct_forward(plan, x, X)
    fcc.fcc_dct_inverse(plan, X, y)
    torch.cuda.synchronize()
    return X.clone(), y.clone()


def _input(n, prec, flags):
    real = bool(flags & fcc.FCC_REAL_INPUT)
    rd = torch.float64 if prec == fcc.FCC_PREC_FP64 else torch.float32
    cd = torch.complex128 if prec == fcc.FCC_PREC_FP64 else torch.complex64
    a = RNG.standard_normal(n ** 3) if real else RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    return torch.from_numpy(a).to(gu.DEV, rd if real else cd)


@pytest.mark.parametrize("n,prec,flags", CASES)
def test_single(n, prec, flags):
    x = _input(n, prec, flags)
    X0, y0 = _round_trip(n, prec, flags, x)
    os.environ["FCC_POISON_SCRATCH"] = "1"
    try:
        X1, y1 = _round_trip(n, prec, flags, x)
    finally:
        os.environ.pop("FCC_POISON_SCRATCH", None)
    assert not torch.isnan(X1).any() and not torch.isnan(y1).any()
    assert torch.equal(X0, X1) and torch.equal(y0, y1)


def test_batched():
    ns = [8, 16, 32, 64, 16, 32]
    xs = [_input(n, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT) for n in ns]

    def run():
        plans = [fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_SPLIT_BF16 if n == 8 else fcc.FCC_PREC_FP32,
                                  flags=fcc.FCC_REAL_INPUT | (fcc.FCC_FOLD_BASE if n == 64 else 0)) for n in ns]
        outs = [torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV) for n in ns]
        back = [torch.empty_like(x) for x in xs]
        fcc.fcc_dct_batched(plans, xs, outs, 1)
        fcc.fcc_dct_batched(plans, outs, back, -1)
        torch.cuda.synchronize()
        fcc.fcc_dct_batched_release()
        return outs, back

    o0, b0 = run()
    os.environ["FCC_POISON_SCRATCH"] = "1"
    try:
        o1, b1 = run()
    finally:
        os.environ.pop("FCC_POISON_SCRATCH", None)
    for i in range(len(ns)):
        assert torch.equal(o0[i], o1[i]) and torch.equal(b0[i], b1[i]), (i, ns[i])
