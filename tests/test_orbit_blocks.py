"""The orbit-block templates of the basis change reproduce the derived gather
tables of B_nl and C_nl exactly (Sec. IV-B, eq. FastAlgorithm; B_n derived
from Prop. 1 (iii), (iv), (vi) and the skew ideal of Sec. IV-A).

The templates are read off the tables of one small node size (32 for
nl >= 16) and the orbits of W on the cube grid mod m are classified into
them; expanding them over every orbit must give every row of the tables of
the target size, entry for entry (source index and exact coefficient
polynomial).  Host logic only: no GPU is used."""
import numpy as np
import pytest

import paper_1807_10058_amd as fcc

FIXED = [(0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0), (1, 0, 1)]  # monomials 1, c3, c1, c2, c1 c3


def _table_polys(T):
    mono = [tuple(int(v) for v in r) for r in T["mono"]]
    out = np.zeros((T["npoly"], 5))
    for q, e in enumerate(mono):
        out[:, FIXED.index(e)] = T["poly"][:, q]
    return np.rint(out * 144).astype(np.int64)


def _poly_ids(keys, intern):
    return np.array([intern.setdefault(tuple(k), len(intern)) for k in keys], dtype=np.int64)


def _expand_tables(T, side, intern):
    nl = T["nl"]
    rp, src, pid = T[side + "_rowptr"], T[side + "_src"], T[side + "_pid"]
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    flat = ((src >> 20) * nl + ((src >> 10) & 1023)) * nl + (src & 1023)
    pk = _poly_ids(_table_polys(T), intern)[pid]
    return rows, flat, pk


def _expand_blocks(B, side, intern):
    nl, m = B["nl"], B["m"]
    G = B["group"]
    pk_of = _poly_ids(np.rint(B["poly"] * 144).astype(np.int64), intern)
    R, S, P = [], [], []
    for t in B["templ"]:
        rep = t["rep"]
        if rep.size == 0:
            continue
        p0 = np.stack([rep >> 20, (rep >> 10) & 1023, rep & 1023], -1)
        q = np.stack([(p0 @ G[w].T) % m for w in t["w"]])  # nc x R x 3 cubes of every orbit
        rp, ent = t[side + "_rowptr"], t[side + "_ent"]
        for r in range(len(rp) - 1):
            j, f = divmod(r, 8)
            fo = np.array([(f >> 2) & 1, (f >> 1) & 1, f & 1])
            for e in ent[rp[r]:rp[r + 1]]:
                s, pid = int(e) >> 8, int(e) & 255
                j2, f2 = divmod(s, 8)
                fo2 = np.array([(f2 >> 2) & 1, (f2 >> 1) & 1, f2 & 1])
                if side == "b":   # row: position f + 2 q_j; source q_j2 + m f2
                    row = ((q[j, :, 0] * m + q[j, :, 1]) * m + q[j, :, 2]) * 8 + f
                    k = q[j2] + m * fo2
                else:             # row: kappa = q_j + m f; source f2 + 2 q_j2
                    kap = q[j] + m * fo
                    row = (((kap[:, 0] >> 1) * m + (kap[:, 1] >> 1)) * m + (kap[:, 2] >> 1)) * 8 + \
                        ((kap[:, 0] & 1) * 4 + (kap[:, 1] & 1) * 2 + (kap[:, 2] & 1))
                    k = 2 * q[j2] + fo2
                R.append(row)
                S.append((k[:, 0] * nl + k[:, 1]) * nl + k[:, 2])
                P.append(np.full(len(row), pk_of[pid]))
    return np.concatenate(R), np.concatenate(S), np.concatenate(P)


def _canon(rows, flat, pk):
    o = np.lexsort((pk, flat, rows))
    return rows[o], flat[o], pk[o]


@pytest.mark.parametrize("nl", [4, 8, 16, 32, 64, 128])
def test_orbit_templates_expand_to_the_tables(nl):
    T = fcc.fcc_asp_tables(nl)
    B = fcc.fcc_asp_orbit_blocks(nl)
    m = nl // 2
    # every cube lies in exactly one orbit
    covered = sum(t["nc"] * len(t["rep"]) for t in B["templ"])
    assert covered == m ** 3
    assert len(B["templ"]) <= 8
    for side in ("b", "c"):
        intern = {}
        a = _canon(*_expand_tables(T, side, intern))
        b = _canon(*_expand_blocks(B, side, intern))
        assert len(a[0]) == len(b[0]), (side, len(a[0]), len(b[0]))
        for x, y in zip(a, b):
            assert np.array_equal(x, y), side


def test_orbit_templates_are_shared_across_sizes():
    """For nl >= 16 the same eight templates serve every node size."""
    ref = fcc.fcc_asp_orbit_blocks(32)
    for nl in (16, 256, 512):
        B = fcc.fcc_asp_orbit_blocks(nl)
        assert B["npoly"] == ref["npoly"] and np.array_equal(B["poly"], ref["poly"])
        assert [t["nc"] for t in B["templ"]] == [t["nc"] for t in ref["templ"]]
        assert sum(t["nc"] * len(t["rep"]) for t in B["templ"]) == B["m"] ** 3
