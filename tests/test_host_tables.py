"""Host logic: the basis-change tables the plan derives (product rule,
dominant map, skew-ideal reduction) satisfy the factorisation identity of
Sec. IV-B eq. FastAlgorithm against the oracle's dense matrices:

    F_nl(phi) C_nl(phi) = P (+)_i F_m((phi+i)/2) (DCT_2(phi) (x) I),   B C = I,

in the interleaved layout the kernels use (node-local position i + 2k holds
child i's entry k).  No GPU needed: the tables are read through the C ABI
introspection call and applied with numpy.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import paper_1807_10058_amd as fcc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

E3 = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
PHI0 = (1 / 8, 0, 3 / 8)


def unpack(s):
    return (s >> 20), (s >> 10) & 1023, s & 1023


def tables_as_matrices(nl, phi):
    t = fcc.fcc_asp_tables(nl)
    m = t["m"]
    c = np.array([oracle.T(e, phi) for e in E3])
    mono = np.array([np.prod(c ** np.array(e)) for e in t["mono"]])
    coef = t["poly"] @ mono
    N = nl ** 3
    flat = lambda x, y, z: (x * nl + y) * nl + z
    B = np.zeros((N, N), complex)
    C = np.zeros((N, N), complex)
    for cube, (a, b, cc) in enumerate(itertools.product(range(m), repeat=3)):
        for f, (d0, d1, d2) in enumerate(itertools.product(range(2), repeat=3)):
            r = cube * 8 + f
            pos = flat(d0 + 2 * a, d1 + 2 * b, d2 + 2 * cc)
            for e in range(t["b_rowptr"][r], t["b_rowptr"][r + 1]):
                B[pos, flat(*unpack(int(t["b_src"][e])))] += coef[t["b_pid"][e]]
            # inverse rows: kappa = i + 2 abc with i = (d0,d1,d2)
            for e in range(t["c_rowptr"][r], t["c_rowptr"][r + 1]):
                C[pos, flat(*unpack(int(t["c_src"][e])))] += coef[t["c_pid"][e]]
    return B, C


def rhs(nl, phi):
    m = nl // 2
    D = oracle.matrix(2, phi)
    N = nl ** 3
    R = np.zeros((N, N), complex)
    flat = lambda v: (v[0] * nl + v[1]) * nl + v[2]
    P2 = list(itertools.product(range(2), repeat=3))
    Pm = list(itertools.product(range(m), repeat=3))
    for ii, i in enumerate(P2):
        Fm = oracle.matrix(m, tuple((np.array(phi) + i) / 2))
        for kk, k in enumerate(Pm):
            row = flat(np.array(i) + 2 * np.array(k))
            for aa, ab in enumerate(Pm):
                for dd, de in enumerate(P2):
                    R[row, flat(np.array(de) + 2 * np.array(ab))] += Fm[kk, aa] * D[ii, dd]
    return R


@pytest.mark.parametrize("nl", [2, 4, 8])
@pytest.mark.parametrize("phi", [PHI0, (0.31, 0.07, 0.23), tuple((np.array(PHI0) + (1, 0, 1)) / 2)])
def test_factorisation_identity(nl, phi):
    B, C = tables_as_matrices(nl, phi)
    N = nl ** 3
    assert np.abs(B @ C - np.eye(N)).max() < 1e-11
    F = oracle.matrix(nl, phi)
    R = rhs(nl, phi)
    assert np.abs(F @ C - R).max() < 1e-12 * max(1, np.abs(R).max())


def test_table_statistics_and_monomials():
    """Sparsity the derivation should reach (O(nl^3) entries, Sec. IV-B) and the
    coefficient polynomials' monomials {1, c3, c1, c2, c1 c3}."""
    prev = 0
    for nl in (4, 8, 16, 32):
        t = fcc.fcc_asp_tables(nl)
        nnz_b = t["b_rowptr"][-1] / nl ** 3
        nnz_c = t["c_rowptr"][-1] / nl ** 3
        assert 3 < nnz_b < 13 and 3 < nnz_c < 10
        assert nnz_b >= prev
        prev = nnz_b
        assert {tuple(v) for v in t["mono"]} <= {(0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0), (1, 0, 1)}
    t2 = fcc.fcc_asp_tables(2)
    assert t2["b_rowptr"][-1] == 8 and t2["c_rowptr"][-1] == 8


def test_derivation_is_identical_across_processes():
    # the parallel derivation interns polynomials in a thread-timing dependent
    # order; the stored coefficients and ids must not depend on it
    import hashlib
    import subprocess
    import sys
    code = ("import hashlib, sys; sys.path.insert(0, %r)\n"
            "import paper_1807_10058_amd as f\n"
            "h = hashlib.sha1()\n"
            "for nl in (16, 32):\n"
            "    t = f.fcc_asp_tables(nl)\n"
            "    for k in ('poly', 'b_src', 'b_pid', 'c_src', 'c_pid'): h.update(t[k].tobytes())\n"
            "print(h.hexdigest())\n") % ROOT
    outs = {subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True).stdout
            for _ in range(4)}
    assert len(outs) == 1, outs


@pytest.mark.parametrize("nl", [8, 32, 64])
def test_tables_are_block_diagonal_over_cube_orbits(nl):
    """The blocks the clustered gather map orders by.  B: cubes whose rows
    share a source, checked against connected components of the cube-source
    graph (scipy), at most 24 cubes (|W|) and 24 for most cubes; every source
    is read by one block.  C = B^{-1}: row kappa reads only positions of the
    block that reads kappa in B."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    t = fcc.fcc_asp_tables(nl)
    m = t["m"]
    blk, kblk = t["cube_block"], t["kappa_block"]

    def flat(s):
        return (s >> 20) * nl * nl + ((s >> 10) & 1023) * nl + (s & 1023)

    rp, src = t["b_rowptr"], t["b_src"]
    cube = np.repeat(np.arange(8 * m ** 3), np.diff(rp)) // 8
    k = flat(src)
    g = coo_matrix((np.ones(len(k)), (cube, m ** 3 + k)), shape=(m ** 3 + nl ** 3,) * 2)
    _, lab = connected_components(g, directed=False)
    lab = lab[:m ** 3]
    pairs = set(zip(lab.tolist(), blk.tolist()))
    assert len(pairs) == len(set(lab.tolist())) == len(set(blk.tolist()))
    first = {}
    for c, b in enumerate(blk.tolist()):
        first.setdefault(b, c)
    assert all(first[b] == b for b in first)  # id = smallest cube of the block
    sizes = np.bincount(blk, minlength=m ** 3)
    sizes = sizes[sizes > 0]
    assert sizes.max() <= 24
    if nl >= 32:
        assert (sizes == 24).sum() * 24 > 0.6 * m ** 3
    # every source is read, by exactly the block kappa_block names
    assert (kblk >= 0).all()
    assert np.array_equal(kblk[k], blk[cube])
    # C rows: kappa = i + 2 abc reads positions def + 2 abc' of block kblk[kappa]
    rp, src = t["c_rowptr"], t["c_src"]
    row = np.repeat(np.arange(8 * m ** 3), np.diff(rp))
    c, i = row // 8, row % 8
    a, b, cc = c // (m * m), (c // m) % m, c % m
    kap = (2 * a + (i >> 2)) * nl * nl + (2 * b + ((i >> 1) & 1)) * nl + (2 * cc + (i & 1))
    x, y, z = src >> 20, (src >> 10) & 1023, src & 1023
    pc = ((x >> 1) * m + (y >> 1)) * m + (z >> 1)
    assert np.array_equal(blk[pc], kblk[kap])
