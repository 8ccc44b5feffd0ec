"""TEST INFRASTRUCTURE ONLY: independent full-volume FP64 reference.

Not the paper's algorithm.  It follows from the explicit matrix of the
transform (Sec. IV-A, eq. SU4ChebyshevTransformExplicitForm) by exchanging the
two sums: with lambda = g k,

    X[j] = sum_k x[k] (1/24) sum_g exp(2 pi i lambda.(rst + j)/n)
         = sum_{mu in [0,n)^3} Fh[mu] exp(2 pi i mu.j / n),
    Fh[mu] = (1/24) sum_{(k,g): g k = mu mod n} x[k] exp(2 pi i (g k).rst / n),

i.e. a twiddled fold onto the n-torus followed by an unnormalised inverse
3-D DFT.  It shares nothing with the direct oracle except the group, which it
rebuilds itself, and is checked against the direct oracle at small n.
"""
import numpy as np

from . import DEFAULT_RST


def _group():
    s = [np.array([[-1, 0, 0], [1, 1, 0], [0, 0, 1]]),
         np.array([[1, 1, 0], [0, -1, 0], [0, 1, 1]]),
         np.array([[1, 0, 0], [0, 1, 1], [0, 0, -1]])]
    out = [np.eye(3, dtype=np.int64)]
    keys = {out[0].tobytes()}
    i = 0
    while i < len(out):
        for g in s:
            h = g @ out[i]
            if h.tobytes() not in keys:
                keys.add(h.tobytes())
                out.append(h)
        i += 1
    return out


def fold_forward(x, n, rst=DEFAULT_RST):
    rst = np.asarray(rst, dtype=np.float64)
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    k = np.stack(np.meshgrid(*([np.arange(n)] * 3), indexing="ij"), -1).reshape(-1, 3)
    Fh = np.zeros((n, n, n), dtype=np.complex128)
    for g in _group():
        lam = k @ g.T
        tw = np.exp(2j * np.pi * (lam @ rst) / n)
        mu = np.mod(lam, n)
        np.add.at(Fh, (mu[:, 0], mu[:, 1], mu[:, 2]), x * tw / 24.0)
    return (np.fft.ifftn(Fh) * n ** 3).reshape(-1)
