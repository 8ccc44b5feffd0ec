"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them retypes the oracle's own
formula: they compare it with a different statement in the paper (power form,
x/y/z parametrisation, sigma/tau/rho, Lemma 1 roots of unity), with identities
of Prop. 1, with an independent fold+FFT evaluation, or with high-precision
mpmath arithmetic.
"""
import itertools

import mpmath
import numpy as np
import pytest

import oracle
from oracle import fold_ref
from tests.conftest import load_golden

RNG = np.random.default_rng(12345)
E3 = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def uvw(theta):
    return [np.exp(2j * np.pi * t) for t in theta]


def test_group_order_and_generators():
    """Sec. III eq. GeneratorMatricesS4: three generators, 24 permutations."""
    G = oracle.group()
    assert G.shape == (24, 3, 3)
    assert len({g.tobytes() for g in G}) == 24
    gens = [np.array(r).reshape(3, 3) for r in load_golden("s4_generators.txt")]
    keys = {g.tobytes() for g in G}
    for s in gens:
        assert s.astype(np.int64).tobytes() in keys
    for g in G:
        assert round(abs(np.linalg.det(g))) == 1
        # closed under products
        for h in G[:3]:
            assert (g @ h).tobytes() in keys


def test_coxeter_relations():
    """The generators are involutions with (s1 s2)^3 = (s2 s3)^3 = (s1 s3)^2 = 1.

    Sec. III prints (s1 s2)^2 = 1 and (s1 s3)^3 = 1; those printed forms do not
    hold for the printed matrices (the S_4 Coxeter relations are the ones above),
    which only matters for presentation: the closure has 24 elements either way."""
    s1, s2, s3 = [np.array(r).reshape(3, 3) for r in load_golden("s4_generators.txt")]
    I = np.eye(3, dtype=int)
    mp = np.linalg.matrix_power
    for s in (s1, s2, s3):
        assert (s @ s == I).all()
    assert (mp(s1 @ s2, 3) == I).all() and (mp(s2 @ s3, 3) == I).all()
    assert (mp(s1 @ s3, 2) == I).all()
    assert not (mp(s1 @ s2, 2) == I).all()
    assert not (mp(s1 @ s3, 3) == I).all()


def test_power_form_matches_orbit_sum():
    """Sec. III eq. A3PowerForm (24 printed monomials) equals Definition 1."""
    terms = [np.array(r).reshape(3, 3) for r in load_golden("a3_power_form.txt")]
    assert len(terms) == 24
    for _ in range(40):
        k = RNG.integers(-4, 9, 3)
        th = RNG.uniform(0, 1, 3)
        u = uvw(th)
        val = sum(u[0] ** (t[0] @ k) * u[1] ** (t[1] @ k) * u[2] ** (t[2] @ k) for t in terms) / 24
        assert abs(oracle.T(k, th) - val) < 1e-13


def test_xyz_parametrisation():
    """Sec. III: x, y, z in terms of u, v, w equal T_100, T_010, T_001 (Prop. 1 ii)."""
    for _ in range(20):
        th = RNG.uniform(0, 1, 3)
        u, v, w = uvw(th)
        x = (u + v / u + w / v + 1 / w) / 4
        y = (1 / v + v + u / w + v / (u * w) + w / u + u * w / v) / 6
        z = (1 / u + u / v + v / w + w) / 4
        for e, ref in zip(E3, (x, y, z)):
            assert abs(oracle.T(e, th) - ref) < 1e-14
        assert abs(np.conj(x) - z) < 1e-14 and abs(y.imag) < 1e-14


def _sigma_tau_rho(r, s, t):
    e = lambda a: np.exp(2j * np.pi * a)
    sig = (e(r) + e(s - r) + e(-t) + e(t - s)) / 4
    tau = (e(-s) + e(s) + e(r - t) + e(s - r - t) + e(t - r) + e(r - s + t)) / 6
    rho = (e(-r) + e(r - s) + e(s - t) + e(t)) / 4
    return sig, tau, rho


def test_skew_auxiliary_functions():
    """Sec. IV-A: sigma, tau, rho are x, y, z at (r,s,t) and all vanish at (1/8,0,3/8)."""
    for _ in range(20):
        rst = RNG.uniform(0, 1, 3)
        for e, v in zip(E3, _sigma_tau_rho(*rst)):
            assert abs(oracle.T(e, rst) - v) < 1e-14
    for v in _sigma_tau_rho(1 / 8, 0, 3 / 8):
        assert abs(v) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8])
def test_lemma1_common_zeros(n):
    """Lemma 1: the sample points are (w_{8n}^{1+8i}, w_n^j, w_{8n}^{3+8k}),
    T_{n00}, T_{0n0}, T_{00n} vanish there, and the n^3 points are distinct."""
    th = oracle.sample_points(n)
    idx = list(itertools.product(range(n), repeat=3))
    w8n = np.exp(2j * np.pi / (8 * n))
    wn = np.exp(2j * np.pi / n)
    xyz = []
    for (i, j, k), t in zip(idx, th):
        u, v, w = uvw(t)
        assert abs(u - w8n ** (1 + 8 * i)) < 1e-13
        assert abs(v - wn ** j) < 1e-13
        assert abs(w - w8n ** (3 + 8 * k)) < 1e-13
        for e in E3:
            assert abs(oracle.T(tuple(n * np.array(e)), t)) < 1e-13
        xyz.append([oracle.T(e, t) for e in E3])
    xyz = np.array(xyz)
    d = np.abs(xyz[:, None, :] - xyz[None, :, :]).max(-1) + np.eye(n ** 3)
    assert d.min() > 1e-6


def test_matrix_orientation_and_T0():
    """Definition 2 / explicit form: rows are sample points, columns basis T_k;
    T_0 = 1 (Prop. 1 i) gives an all-ones first column, and the first row is
    T_k at theta_0."""
    n = 3
    F = oracle.matrix(n)
    assert np.allclose(F[:, 0], 1.0, atol=1e-15)
    th0 = oracle.sample_points(n)[0]
    k = [(a, b, c) for a in range(n) for b in range(n) for c in range(n)]
    assert max(abs(F[0, q] - oracle.T(kk, th0)) for q, kk in enumerate(k)) < 1e-15
    assert not np.allclose(F[0, :], 1.0)
    assert np.allclose(oracle.matrix(1), [[1.0]])


def test_weyl_invariance_product_rule_semigroup():
    """Prop. 1 (iii) W-invariance, (iv) product rule with the orbit {a + g b},
    (vi) semigroup T_{l k}(theta) = T_k(l theta)."""
    G = oracle.group()
    for _ in range(15):
        th = RNG.uniform(0, 1, 3)
        a = RNG.integers(-3, 6, 3)
        b = RNG.integers(-3, 6, 3)
        Ta = oracle.T(a, th)
        for g in G[:: 5]:
            assert abs(oracle.T(g @ a, th) - Ta) < 1e-13
        lhs = Ta * oracle.T(b, th)
        rhs = sum(oracle.T(a + g @ b, th) for g in G) / 24
        assert abs(lhs - rhs) < 1e-13
        l = int(RNG.integers(2, 5))
        assert abs(oracle.T(l * a, th) - oracle.T(a, l * th)) < 1e-13


def test_conjugation_symmetry():
    """Sec. III: x and z are conjugate, y real, hence conj T_{j,k,p} = T_{p,k,j};
    for the transform matrix every row has a conjugate partner row."""
    for _ in range(20):
        th = RNG.uniform(0, 1, 3)
        j, k, p = RNG.integers(0, 7, 3)
        assert abs(np.conj(oracle.T((j, k, p), th)) - oracle.T((p, k, j), th)) < 1e-13
    for n in (2, 4):
        F = oracle.matrix(n)
        C = np.conj(F)
        d = np.abs(F[:, None, :] - C[None, :, :]).max(-1)
        assert (d.min(1) < 1e-12).all()


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("rst", [(1 / 8, 0, 3 / 8), (0.31, 0.07, 0.23)])
def test_independent_fold_fft_matches(n, rst):
    """The fold+FFT evaluation (a different algorithm) reproduces the direct sum."""
    x = RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    X = oracle.forward(x, n, rst)
    Y = fold_ref.fold_forward(x, n, rst)
    assert np.abs(X - Y).max() <= 1e-13 * max(1.0, np.abs(X).max())


def test_sampled_rows_match_fold_at_16():
    n = 16
    x = RNG.uniform(-1, 1, n ** 3)
    rows = RNG.choice(n ** 3, 64, replace=False)
    X = oracle.forward_rows(x, n, rows)
    Y = fold_ref.fold_forward(x, n)[rows]
    assert np.abs(X - Y).max() <= 1e-12 * np.abs(Y).max()


def test_entries_against_mpmath():
    """A few entries in 30-digit arithmetic from the printed power form (both the
    exact-phase path at (1/8,0,3/8) and the general path at another (r,s,t))."""
    terms = [np.array(r).reshape(3, 3) for r in load_golden("a3_power_form.txt")]
    mpmath.mp.dps = 30
    for rst in ((mpmath.mpf(1) / 8, 0, mpmath.mpf(3) / 8), (mpmath.mpf("0.31"), mpmath.mpf("0.07"), mpmath.mpf("0.23"))):
        n = 5
        F = oracle.matrix(n, tuple(float(v) for v in rst))
        for _ in range(12):
            j = RNG.integers(0, n, 3)
            k = RNG.integers(0, n, 3)
            th = [(rst[d] + int(j[d])) / n for d in range(3)]
            val = mpmath.mpc(0)
            for t in terms:
                e = t @ k
                val += mpmath.expjpi(2 * (e[0] * th[0] + e[1] * th[1] + e[2] * th[2]))
            val /= 24
            got = F[(j[0] * n + j[1]) * n + j[2], (k[0] * n + k[1]) * n + k[2]]
            assert abs(complex(val) - got) < 5e-15


@pytest.mark.parametrize("n", [2, 4, 8])
def test_invertible_and_roundtrip(n):
    """Lemma 2: distinct zeros make the transform invertible; the dense inverse
    satisfies forward(inverse(X)) = X to 1e-12 (the n=4 round-trip tolerance)."""
    F = oracle.matrix(n)
    assert np.linalg.cond(F) < 20
    X = RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    x = oracle.inverse(X, n)
    assert np.abs(oracle.forward(x, n) - X).max() <= 1e-12 * np.abs(X).max()


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("rst", [(1 / 8, 0, 3 / 8), (0.31, 0.07, 0.23)])
def test_fold_inverse_matches_dense_inverse(n, rst):
    """The fold inverse (DFT, then per-orbit solves of the fold) equals the
    oracle's dense LU inverse of the explicit matrix (Sec. IV-A, Lemma 2)."""
    X = RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    x = oracle.inverse(X, n, rst)
    y = fold_ref.fold_inverse(X, n, rst)
    assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_fold_inverse_orbits_partition_the_torus():
    """The blocks of the fold are the orbits of W on the n-torus: every point
    lies in one, g k mod n stays in its orbit, and no orbit has more than 24 points."""
    n = 16
    rep, order = fold_ref.torus_orbits(n)
    k = np.stack(np.meshgrid(*([np.arange(n)] * 3), indexing="ij"), -1).reshape(-1, 3)
    for g in oracle.group():
        img = np.mod(k @ g.T, n)
        assert np.array_equal(rep[(img[:, 0] * n + img[:, 1]) * n + img[:, 2]], rep)
    assert np.bincount(np.unique(rep, return_counts=True)[1]).nonzero()[0].max() <= 24
    assert np.array_equal(np.sort(order), np.arange(n ** 3))


@pytest.mark.parametrize("n", [16, 32])
def test_fold_inverse_undoes_the_direct_forward(n):
    """fold_inverse(forward(x)) = x, with forward from the direct sum at n = 16
    and from sampled direct rows plus the fold at n = 32; sampled points alone
    give the same values as the full solve."""
    x = RNG.standard_normal(n ** 3)
    X = oracle.forward(x, n) if n == 16 else fold_ref.fold_forward(x, n)
    if n == 32:
        rows = RNG.choice(n ** 3, 16, replace=False)
        assert np.abs(oracle.forward_rows(x, n, rows) - X[rows]).max() <= 1e-12 * np.abs(X).max()
    y = fold_ref.fold_inverse(X, n)
    assert np.abs(y - x).max() <= 1e-12 * np.abs(x).max()
    pts = RNG.choice(n ** 3, 40, replace=False)
    assert np.array_equal(fold_ref.fold_inverse(X, n, points=pts), y[pts])


@pytest.mark.parametrize("n", [2, 4, 8])
def test_transposed_rows_are_the_matrix_transpose(n):
    """The transposed reading X_T = F^T x (the literal row/column labels after
    eq. SU4ChebyshevTransformExplicitForm), entry by entry from the orbit sum,
    equals the transpose of the direct matrix."""
    F = oracle.matrix(n)
    x = RNG.standard_normal(n ** 3) + 1j * RNG.standard_normal(n ** 3)
    ks = RNG.choice(n ** 3, min(16, n ** 3), replace=False)
    assert np.abs(oracle.transposed_rows(x, n, ks) - (F.T @ x)[ks]).max() <= 1e-12 * np.abs(F.T @ x).max()


@pytest.mark.parametrize("n", [2, 4, 8])
def test_hermitian_pairing_of_real_spectra(n):
    """For real input, X[j'] = conj X[j] with j' = -g^T j mod n for the one g of W
    with g^T rst = -rst mod 1 (realness of T, Sec. III: conj T_(j,k,p) = T_(p,k,j));
    the pairing is an involution with n^2 fixed points."""
    G = oracle.group()
    rst = np.array(oracle.DEFAULT_RST)
    gs = [g for g in G if np.allclose(np.mod(-g.T @ rst - rst + 0.5, 1.0), 0.5)]
    assert len(gs) == 1
    g = gs[0]
    c = np.rint(-g.T @ rst - rst).astype(int)
    j = np.stack(np.unravel_index(np.arange(n ** 3), (n, n, n)), -1)
    q = np.mod(-(j @ g) + c, n)
    jp = (q[:, 0] * n + q[:, 1]) * n + q[:, 2]
    assert np.array_equal(jp[jp], np.arange(n ** 3))
    assert (jp == np.arange(n ** 3)).sum() == n * n
    x = RNG.standard_normal(n ** 3)
    X = oracle.forward(x, n)
    assert np.abs(X[jp] - np.conj(X)).max() <= 1e-12 * np.abs(X).max()
