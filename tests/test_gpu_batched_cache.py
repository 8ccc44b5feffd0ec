"""fcc_dct_batched keeps at most a few recorded graphs (least recently used
freed first) and fcc_dct_batched_release frees them all: calls with fresh
buffers every time must not grow device memory without bound."""
import numpy as np
import pytest
import torch

import paper_1807_10058_amd as fcc

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_fresh_buffers_do_not_grow_memory():
    ns = [32, 64, 32, 16]
    plans = {n: fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT) for n in set(ns)}
    xs = [torch.from_numpy(np.random.default_rng(n).standard_normal(n ** 3).astype(np.float32)).to(gu.DEV)
          for n in ns]
    fcc.fcc_dct_batched_release()
    base = _free()
    after = []
    for it in range(12):
        # a new output set each call: a new graph-cache key each time
        outs = [torch.empty(n ** 3 + 64 * it, dtype=torch.complex64, device=gu.DEV)[: n ** 3] for n in ns]
        fcc.fcc_dct_batched([plans[n] for n in ns], xs, outs, 1)
        after.append(_free())
        del outs
    # the cache is bounded: memory taken after the 12th call is no more than after the 6th (plus slack)
    slack = 64 << 20
    assert after[-1] >= after[5] - slack, (after[5], after[-1])
    fcc.fcc_dct_batched_release()
    torch.cuda.empty_cache()
    assert _free() >= base - slack
