"""Helpers for the GPU parity tests: run the HIP path through the C ABI on
torch device buffers and measure errors against the oracle."""
import numpy as np
import torch

import paper_1807_10058_amd as fcc

DEV = torch.device("cuda:0")


def cdtype(prec):
    return torch.complex128 if prec == fcc.FCC_PREC_FP64 else torch.complex64


def rdtype(prec):
    return torch.float64 if prec == fcc.FCC_PREC_FP64 else torch.float32


def forward(x, n, prec=fcc.FCC_PREC_FP64, rst=None, flags=0):
    """x: numpy real or complex array of n^3 values."""
    real = not np.iscomplexobj(x)
    flags |= fcc.FCC_REAL_INPUT if real else 0
    plan = fcc.fcc_dct_plan(n, rst=rst, prec=prec, flags=flags)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV, rdtype(prec) if real else cdtype(prec))
    Xt = torch.empty(n ** 3, dtype=cdtype(prec), device=DEV)
    fcc.fcc_dct_forward(plan, xt, Xt)
    torch.cuda.synchronize()
    return Xt.cpu().numpy().astype(np.complex128), plan


def inverse(X, n, prec=fcc.FCC_PREC_FP64, rst=None, flags=0, real_out=False):
    flags |= fcc.FCC_REAL_INPUT if real_out else 0
    plan = fcc.fcc_dct_plan(n, rst=rst, prec=prec, flags=flags)
    Xt = torch.from_numpy(np.ascontiguousarray(X)).to(DEV, cdtype(prec))
    out = torch.empty(n ** 3, dtype=rdtype(prec) if real_out else cdtype(prec), device=DEV)
    fcc.fcc_dct_inverse(plan, Xt, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64 if real_out else np.complex128)


def maxrel(y, ref):
    return float(np.abs(np.asarray(y) - np.asarray(ref)).max() / np.abs(ref).max())


def sample_rows(n, count, seed):
    """Seeded sample of flat output indices, always with the corners and index 0."""
    rng = np.random.default_rng(seed)
    corners = [((a * n + b) * n + c) for a in (0, n - 1) for b in (0, n - 1) for c in (0, n - 1)]
    rows = set(int(v) for v in rng.choice(n ** 3, size=min(count, n ** 3), replace=False)) | set(corners)
    return np.array(sorted(rows), dtype=np.int64)
