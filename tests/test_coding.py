"""Pins of the spectrum quantiser reference (block-wise coding, the application
of Sec. I and Sec. V) against its definition: threshold on the magnitude,
round-half-to-even codes, saturation, dequantisation; and the rebuilt blocks
against the direct forward (host only)."""
import numpy as np

import oracle
from oracle import coding


def test_threshold_rounding_and_saturation():
    X = np.array([3 + 4j, 2.9 + 4j, 0.5 + 0j, 1.5 - 2.5j, 1e6 + 0j, -1e6 + 0j], dtype=np.complex64)
    codes, Xq, kept = coding.quantise(X, threshold=5.0, step=1.0)
    # |3+4i| = 5 is kept (>=), |2.9+4i| < 5 is not
    assert codes[0].tolist() == [3, 4] and codes[1].tolist() == [0, 0]
    assert codes[2].tolist() == [0, 0]
    codes, Xq, kept = coding.quantise(X, threshold=0.0, step=1.0)
    assert codes[2].tolist() == [0, 0]                      # rint(0.5) = 0 (half to even)
    assert codes[3].tolist() == [2, -2]                     # rint(1.5) = 2, rint(-2.5) = -2
    assert codes[4].tolist() == [32767, 0] and codes[5].tolist() == [-32768, 0]
    assert kept == 6
    assert np.array_equal(Xq, (codes[:, 0] + 1j * codes[:, 1]).astype(np.complex64))


def test_rebuild_inverts_the_forward():
    n = 4
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (3, n ** 3))
    X = np.stack([oracle.forward(v, n) for v in x])
    y = coding.rebuild(X, n)
    assert np.abs(y - x).max() <= 1e-12
