"""TEST INFRASTRUCTURE ONLY: plain reference of the spectrum quantiser used for
block-wise volumetric coding (the application motivating the transform, Sec. I
and Sec. V of the paper), and of the rebuilt blocks.

For a complex coefficient X = (re, im), in IEEE FP32 with every operation
rounded once:  keep = re*re + im*im >= threshold^2;  code = keep ?
(rint(re / step), rint(im / step)) : 0, saturated to int16;  Xq = step * code.
Blocks are rebuilt as x = F^{-1} Xq with the oracle's dense matrix F of
Definition 2 (LU solve in FP64).
"""
import numpy as np

from . import matrix


def quantise(X, threshold, step):
    """codes (int16, shape (..., 2)), dequantised Xq (complex64) and the kept count."""
    X = np.asarray(X, dtype=np.complex64)
    re = X.real.astype(np.float32)
    im = X.imag.astype(np.float32)
    t = np.float32(threshold)
    s = np.float32(step)
    m2 = (re * re) + (im * im)          # float32: each product and the sum rounded once
    keep = m2 >= t * t
    cr = np.clip(np.rint(re / s), -32768, 32767).astype(np.int16)
    ci = np.clip(np.rint(im / s), -32768, 32767).astype(np.int16)
    cr[~keep] = 0
    ci[~keep] = 0
    codes = np.stack([cr, ci], -1)
    Xq = (s * cr.astype(np.float32)) + 1j * (s * ci.astype(np.float32))
    return codes, Xq.astype(np.complex64), int(keep.sum())


def rebuild(Xq_blocks, n, rst=None):
    """x = F^{-1} Xq for every block (rows of Xq_blocks), FP64 dense LU."""
    F = matrix(n) if rst is None else matrix(n, rst)
    return np.linalg.solve(F, np.asarray(Xq_blocks, dtype=np.complex128).T).T
