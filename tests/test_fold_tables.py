"""Host-side unfold tables of the fold+FFT variant (FCC_FOLD_FFT), checked on
the CPU without a device: with the library's rows K and per-point indices,

    x[k] = sum_u K[pid[k]][u] exp(-2 pi i (u k).rst / n) Fh[u k mod n],  Fh = DFT_3(X) / n^3,

must return the input of X = fold_ref.fold_forward(x) (the independent FP64
reference of the explicit matrix, Sec. IV-A), for the default skew and another
skew with 8 rst integral; skews with coinciding zeros are refused."""
import numpy as np
import pytest

import paper_1807_10058_amd as fcc
from oracle import fold_ref

RNG = np.random.default_rng(1058)
G = fold_ref._group()  # same closure order as the library's group table


def _unfold(X, n, pid, K, rst):
    N = n ** 3
    Fh = (np.fft.fftn(X.reshape(n, n, n)) / N).reshape(-1)
    k = fold_ref._grid(n)
    x = np.zeros(N, dtype=np.complex128)
    for u, g in enumerate(G):
        uk = k @ g.T
        x += K[pid, u] * np.exp(-2j * np.pi * (uk @ np.asarray(rst)) / n) * Fh[fold_ref._flat(np.mod(uk, n), n)]
    return x


@pytest.mark.parametrize("rst", [(0.125, 0.0, 0.375), (0.625, 0.0, 0.875)])
@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_unfold_inverts_the_fold(n, rst):
    pid, K = fcc.fcc_fold_unfold_tables(n, rst)
    assert pid.max() < len(K) <= 64
    x = RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    X = fold_ref.fold_forward(x, n, rst)
    assert np.abs(_unfold(X, n, pid, K, rst) - x).max() <= 1e-12 * np.abs(x).max()


def test_rows_do_not_grow_with_n():
    counts = [len(fcc.fcc_fold_unfold_tables(n)[1]) for n in (8, 16, 32, 64)]
    assert counts == [counts[0]] * 4


@pytest.mark.parametrize("rst", [(0.0, 0.0, 0.0), (0.125, 0.25, 0.375)])
def test_singular_skews_refused(rst):
    with pytest.raises(fcc.FccError, match="SINGULAR"):
        fcc.fcc_fold_unfold_tables(8, rst)


def test_skew_without_eighths_refused():
    with pytest.raises(fcc.FccError, match="UNSUPPORTED"):
        fcc.fcc_fold_unfold_tables(8, (0.31, 0.07, 0.23))


def test_tables_are_deterministic():
    """n = 32 and 64 build their tables on several host threads; the row
    numbering and values must not depend on thread timing."""
    for n in (32, 64):
        ref = fcc.fcc_fold_unfold_tables(n)
        for _ in range(3):
            pid, K = fcc.fcc_fold_unfold_tables(n)
            assert np.array_equal(pid, ref[0]) and np.array_equal(K, ref[1])
