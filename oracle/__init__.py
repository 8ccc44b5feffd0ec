"""TEST INFRASTRUCTURE ONLY: the CPU FP64 oracle for the FCC cosine transform.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library.

``fcc_oracle.c`` holds the plain O(N^2) definition (Sec. III Definition 1 for
T_k, Sec. IV-A Definition 2 and eq. SU4ChebyshevTransformExplicitForm for the
transform).  This module wraps it with ctypes and adds:

* ``inverse`` -- the exact inverse of the transform matrix via a dense FP64 LU
  solve (``numpy.linalg.solve``), for n <= 16;
* ``fold_ref`` -- an independent full-volume FP64 reference (see that module).

Index triples are flattened lexicographically, (a,b,c) -> (a*n+b)*n+c; rows of
the transform are sample points j, columns basis indices k.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_fcc_oracle.so")
SRC = os.path.join(HERE, "fcc_oracle.c")
DEFAULT_RST = (1.0 / 8.0, 0.0, 3.0 / 8.0)  # Sec. IV-A, Definition 2

_lib = None


def build(force=False):
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the .so path."""
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        tmp = SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        L = ctypes.CDLL(SO)
        dp = ctypes.POINTER(ctypes.c_double)
        L.fcco_group.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.fcco_T.argtypes = [ctypes.POINTER(ctypes.c_int), dp, dp]
        L.fcco_matrix.argtypes = [ctypes.c_int, dp, dp]
        L.fcco_forward_rows.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_longlong), dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def group():
    """The 24 integer 3x3 matrices of W = <s1, s2, s3> (eq. GeneratorMatricesS4)."""
    buf = np.zeros(64 * 9, dtype=np.int32)
    cnt = lib().fcco_group(buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 64)
    return buf[: 9 * cnt].reshape(cnt, 3, 3).astype(np.int64)


def T(k, theta):
    """T_k(theta) = (1/24) sum_g exp(2 pi i (g k).theta)  (Definition 1)."""
    kk = np.ascontiguousarray(k, dtype=np.int32)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros(2)
    lib().fcco_T(kk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(th), _dp(out))
    return complex(out[0], out[1])


def sample_points(n, rst=DEFAULT_RST):
    """theta_j = ((r,s,t) + j)/n, j in [0,n)^3 lexicographic (Lemma 2)."""
    j = np.stack(np.meshgrid(*([np.arange(n)] * 3), indexing="ij"), -1).reshape(-1, 3)
    return (np.asarray(rst, float)[None, :] + j) / n


def matrix(n, rst=DEFAULT_RST):
    """Dense DCT_{n x n x n}(r,s,t): F[j, k] = T_k(theta_j) (eq. SU4ChebyshevTransformExplicitForm)."""
    N = n ** 3
    F = np.zeros((N, N), dtype=np.complex128)
    r = np.ascontiguousarray(rst, dtype=np.float64)
    if lib().fcco_matrix(n, _dp(r), _dp(F.view(np.float64))) != 0:
        raise MemoryError("oracle matrix")
    return F


def forward_rows(x, n, rows, rst=DEFAULT_RST):
    """X[rows] of the forward transform, each row an O(24 N) sum."""
    xc = np.ascontiguousarray(np.asarray(x).reshape(-1), dtype=np.complex128)
    assert xc.size == n ** 3
    rr = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rr.size, dtype=np.complex128)
    r = np.ascontiguousarray(rst, dtype=np.float64)
    rc = lib().fcco_forward_rows(n, _dp(r), _dp(xc.view(np.float64)), int(rr.size),
                                 rr.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                 _dp(out.view(np.float64)))
    if rc != 0:
        raise MemoryError("oracle rows")
    return out


def forward(x, n, rst=DEFAULT_RST):
    """Full forward transform X = F x by the direct definition."""
    return forward_rows(x, n, np.arange(n ** 3), rst)


def inverse(X, n, rst=DEFAULT_RST):
    """x = F^{-1} X by a dense FP64 LU solve (n <= 16)."""
    if n > 16:
        raise ValueError("dense oracle inverse only for n <= 16")
    return np.linalg.solve(matrix(n, rst), np.asarray(X, dtype=np.complex128).reshape(-1))


def transposed_rows(x, n, kappas, rst=DEFAULT_RST):
    """Entries kappas of the transposed transform (the literal row/column
    reading of eq. SU4ChebyshevTransformExplicitForm): X_T[k] = sum_j T_k(theta_j) x[j],
    each an O(24 N) sum in numpy (T_k written out as the orbit sum of Definition 1)."""
    G = group()
    th = sample_points(n, rst)
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    out = []
    for k in np.asarray(kappas).reshape(-1):
        kv = np.array([k // (n * n), (k // n) % n, k % n])
        Tk = np.exp(2j * np.pi * (th @ (G @ kv).T)).mean(axis=1)
        out.append(Tk @ x)
    return np.array(out)


def num_threads():
    return int(lib().fcco_num_threads())
