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

The inverse runs the two steps backwards: Fh = DFT(X) / n^3, then x = Fold^{-1}
Fh.  Fold only moves k inside its orbit under W acting on the n-torus
(g k mod n), so Fold is block diagonal over those orbits (at most 24 points
each) and every block is solved on its own.
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


def _grid(n):
    return np.stack(np.meshgrid(*([np.arange(n, dtype=np.int64)] * 3), indexing="ij"), -1).reshape(-1, 3)


def _flat(v, n):
    return (v[..., 0] * n + v[..., 1]) * n + v[..., 2]


def fold_forward(x, n, rst=DEFAULT_RST):
    rst = np.asarray(rst, dtype=np.float64)
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    k = _grid(n)
    N = n ** 3
    re = np.zeros(N)
    im = np.zeros(N)
    for g in _group():
        lam = k @ g.T
        v = x * np.exp(2j * np.pi * (lam @ rst) / n) / 24.0
        mu = _flat(np.mod(lam, n), n)
        re += np.bincount(mu, weights=v.real, minlength=N)
        im += np.bincount(mu, weights=v.imag, minlength=N)
    Fh = (re + 1j * im).reshape(n, n, n)
    return (np.fft.ifftn(Fh) * N).reshape(-1)


def torus_orbits(n):
    """Orbits of W on the n-torus: for every point its orbit's smallest flat
    index, and the points sorted by (orbit, flat index)."""
    k = _grid(n)
    rep = _flat(k, n)
    for g in _group():
        rep = np.minimum(rep, _flat(np.mod(k @ g.T, n), n))
    order = np.lexsort((np.arange(n ** 3), rep))
    return rep, order


def fold_inverse(X, n, rst=DEFAULT_RST, points=None):
    """x = DCT_n(rst)^{-1} X through Fh = DFT(X)/n^3 and per-orbit solves of
    Fold x = Fh.  With `points` (flat indices), only the orbits holding them
    are solved and x is returned at those points."""
    rst = np.asarray(rst, dtype=np.float64)
    N = n ** 3
    Fh = (np.fft.fftn(np.asarray(X, dtype=np.complex128).reshape(n, n, n)) / N).reshape(-1)
    rep, order = torus_orbits(n)
    srep = rep[order]
    starts = np.flatnonzero(np.r_[True, srep[1:] != srep[:-1]])
    sizes = np.diff(np.r_[starts, N])
    local = np.empty(N, dtype=np.int64)
    local[order] = np.arange(N) - np.repeat(starts, sizes)
    orbit_of = np.empty(N, dtype=np.int64)
    orbit_of[order] = np.repeat(np.arange(len(starts)), sizes)
    wanted = np.ones(len(starts), dtype=bool)
    if points is not None:
        wanted[:] = False
        wanted[orbit_of[np.asarray(points)]] = True
    x = np.zeros(N, dtype=np.complex128)
    G = _group()
    for s in np.unique(sizes):
        ids = np.flatnonzero((sizes == s) & wanted)
        for c0 in range(0, len(ids), 50000):
            oid = ids[c0:c0 + 50000]
            mem = order[(starts[oid][:, None] + np.arange(s)[None, :]).reshape(-1)]  # members, orbit-major
            kv = np.stack([mem // (n * n), (mem // n) % n, mem % n], -1)
            blk = np.repeat(np.arange(len(oid)), s)
            re = np.zeros(len(oid) * s * s)
            im = np.zeros(len(oid) * s * s)
            for g in G:
                lam = kv @ g.T
                w = np.exp(2j * np.pi * (lam @ rst) / n) / 24.0
                row = local[_flat(np.mod(lam, n), n)]
                idx = (blk * s + row) * s + local[mem]
                re += np.bincount(idx, weights=w.real, minlength=re.size)
                im += np.bincount(idx, weights=w.imag, minlength=im.size)
            A = (re + 1j * im).reshape(len(oid), s, s)
            rhs = Fh[mem].reshape(len(oid), s, 1)
            x[mem] = np.linalg.solve(A, rhs).reshape(-1)
    return x if points is None else x[np.asarray(points)]
