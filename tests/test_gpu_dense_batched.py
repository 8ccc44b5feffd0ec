"""GPU parity of the dense split-precision MFMA path and of batched execution.

The dense path applies the whole DCT_{n x n x n} matrix (n <= 8) to many
blocks with split hi+lo BF16/FP16 operands and FP32 accumulation; the
reference is the oracle's dense FP64 matrix applied with an FP64 matmul (a
library primitive).  Tolerance 1e-4 relative per block (max over blocks).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_10058_amd as fcc
import workloads

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
RNG = np.random.default_rng(77)


def per_block_maxrel(Y, R):
    return float((np.abs(Y - R).max(1) / np.abs(R).max(1)).max())


def dense_forward(blocks, n, prec):
    B = blocks.shape[0]
    plans = [fcc.fcc_dct_plan(n, prec=prec, flags=fcc.FCC_REAL_INPUT)]
    x = torch.from_numpy(blocks).to(gu.DEV)
    X = torch.empty((B, n ** 3), dtype=torch.complex64, device=gu.DEV)
    fcc.fcc_dct_batched(plans * B, [x[b] for b in range(B)], [X[b] for b in range(B)], +1)
    torch.cuda.synchronize()
    return X.cpu().numpy().astype(np.complex128), plans[0], x, X


@pytest.mark.parametrize("prec", [fcc.FCC_PREC_SPLIT_BF16, fcc.FCC_PREC_SPLIT_FP16])
def test_dense_split_n8_quantised_blocks(prec):
    """4096 blocks of 8-bit levels / 255 at n = 8 (the block-coding case)."""
    n = 8
    blocks = workloads.quantised_blocks(4096, n, seed=2)
    X, plan, x, Xt = dense_forward(blocks, n, prec)
    F = oracle.matrix(n)
    R = blocks.astype(np.float64) @ F.T
    assert per_block_maxrel(X, R) <= 1e-4
    # inverse through the same plan (single call on block 0 and batched on all)
    y = torch.empty(n ** 3, dtype=torch.float32, device=gu.DEV)
    fcc.fcc_dct_inverse(plan, Xt[0], y)
    torch.cuda.synchronize()
    assert gu.maxrel(y.cpu().numpy(), blocks[0]) <= 1e-4


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("prec", [fcc.FCC_PREC_SPLIT_BF16, fcc.FCC_PREC_SPLIT_FP16])
def test_dense_split_single_and_complex(n, prec):
    N = n ** 3
    x = (RNG.standard_normal(N) + 1j * RNG.standard_normal(N)).astype(np.complex64)
    plan = fcc.fcc_dct_plan(n, prec=prec, flags=0)
    xt = torch.from_numpy(x).to(gu.DEV)
    Xt = torch.empty(N, dtype=torch.complex64, device=gu.DEV)
    fcc.fcc_dct_forward(plan, xt, Xt)
    yt = torch.empty(N, dtype=torch.complex64, device=gu.DEV)
    fcc.fcc_dct_inverse(plan, Xt, yt)
    torch.cuda.synchronize()
    ref = oracle.forward(x.astype(np.complex128), n)
    assert gu.maxrel(Xt.cpu().numpy(), ref) <= 1e-4
    assert gu.maxrel(yt.cpu().numpy(), x) <= 1e-4


def test_fp32_fast_path_n8_blocks_for_comparison():
    """The plain FP32 fast path on the same n = 8 blocks (the comparison case)."""
    n = 8
    blocks = workloads.quantised_blocks(512, n, seed=2)
    plans = [fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT)]
    x = torch.from_numpy(blocks).to(gu.DEV)
    X = torch.empty((512, n ** 3), dtype=torch.complex64, device=gu.DEV)
    fcc.fcc_dct_batched(plans * 512, [x[b] for b in range(512)], [X[b] for b in range(512)], +1)
    torch.cuda.synchronize()
    R = blocks.astype(np.float64) @ oracle.matrix(n).T
    assert per_block_maxrel(X.cpu().numpy(), R) <= 1e-5


def test_ragged_batched_roundtrip_and_graph_replay():
    """Ragged sizes in one batched call (forward then inverse), replayed three
    times with eager work in between; every replay matches the single calls."""
    ns, xs = workloads.ragged_batch(count=24, seed=4, sizes=(2, 4, 8, 16, 32))
    plans = {n: fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT) for n in set(ns)}
    P = [plans[n] for n in ns]
    ins = [torch.from_numpy(x).to(gu.DEV) for x in xs]
    outs = [torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV) for n in ns]
    # reference: single-volume forward calls
    refs = []
    for n, x in zip(ns, ins):
        o = torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV)
        fcc.fcc_dct_forward(plans[n], x, o)
        refs.append(o)
    torch.cuda.synchronize()
    for rep in range(3):
        for i, x in enumerate(xs):
            ins[i].copy_(torch.from_numpy(x).to(gu.DEV))
        _ = torch.randn(1000, device=gu.DEV).sum()  # unrelated eager work between replays
        fcc.fcc_dct_batched(P, ins, outs, 0)
        torch.cuda.synchronize()
        for i, (n, x) in enumerate(zip(ns, xs)):
            assert gu.maxrel(outs[i].cpu().numpy(), refs[i].cpu().numpy()) <= 1e-6, (rep, i, n)
            assert gu.maxrel(ins[i].cpu().numpy(), x) <= 1e-5, (rep, i, n)
    # forward outputs against the oracle on a few volumes
    for i in range(0, len(ns), 6):
        n = ns[i]
        rows = gu.sample_rows(n, 32, i)
        ref = oracle.forward_rows(xs[i].astype(np.float64), n, rows)
        assert gu.maxrel(outs[i].cpu().numpy()[rows], ref) <= 1e-5


def test_ragged_mixed_precision_batch():
    """The mixed form of the ragged workload in one batched call: n = 8 on the
    split-BF16 dense path, larger n with the top level in FP32.  Forward
    against the oracle and round trip within 1e-4, on two graph replays."""
    ns, xs = workloads.ragged_batch(count=18, seed=4, sizes=(8, 16, 32))
    plans = {}
    for n in set(ns):
        if n <= 8:
            plans[n] = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_SPLIT_BF16, flags=fcc.FCC_REAL_INPUT)
        else:
            plans[n] = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32,
                                        flags=fcc.FCC_REAL_INPUT | fcc.FCC_LEVEL0_FP32)
    P = [plans[n] for n in ns]
    ins = [torch.from_numpy(x).to(gu.DEV) for x in xs]
    outs = [torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV) for n in ns]
    for rep in range(2):
        for i, x in enumerate(xs):
            ins[i].copy_(torch.from_numpy(x).to(gu.DEV))
        fcc.fcc_dct_batched(P, ins, outs, 0)
        torch.cuda.synchronize()
        for i, (n, x) in enumerate(zip(ns, xs)):
            assert gu.maxrel(ins[i].cpu().numpy(), x) <= 1e-4, (rep, i, n)
    for i in range(0, len(ns), 3):
        n = ns[i]
        rows = gu.sample_rows(n, 32, i)
        ref = oracle.forward_rows(xs[i].astype(np.float64), n, rows)
        assert gu.maxrel(outs[i].cpu().numpy()[rows], ref) <= 1e-4, (i, n)


def test_batched_rejects_bad_arguments():
    plan = fcc.fcc_dct_plan(4, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT)
    x = torch.zeros(64, dtype=torch.float32, device=gu.DEV)
    X = torch.zeros(64, dtype=torch.complex64, device=gu.DEV)
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_batched([plan], [x], [X], 3)
    assert e.value.status == 1
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_batched([plan], [x], [x], 1)
    assert e.value.status == 1


def test_dense_rejects_large_n():
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan(16, prec=fcc.FCC_PREC_SPLIT_BF16)
    assert e.value.status == 6
