"""Schedules (fused-tail depth, tile shape and block map of the upper gather
passes) through the C ABI: tile and map choices give bit-identical results,
every tail depth matches the oracle, and the autotuner's choice is what later
plans use."""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_10058_amd as fcc
import workloads

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")


def tuning(tail=(1, 1), tiles=((0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0)), maps=(0, 0, 0, 0), deep=(0, 0)):
    """tiles/maps in the order (fwd L0, fwd L1, inv L0, inv L1); deep = the
    (forward, inverse) map of every level from 2 on."""
    return {"tail_levels": list(tail),
            "tile": [[list(tiles[0]), list(tiles[1])], [list(tiles[2]), list(tiles[3])]],
            "map": [[maps[0], maps[1]] + [deep[0]] * 8, [maps[2], maps[3]] + [deep[1]] * 8]}


N8, N64, SP, BAL, X16, CL = (fcc.FCC_MAP_NODES8, fcc.FCC_MAP_NODES64, fcc.FCC_MAP_SPLIT, fcc.FCC_MAP_BALANCE,
                             fcc.FCC_MAP_XCD16, fcc.FCC_MAP_CLUSTER)
SCHEDULES = [
    tuning(),
    tuning(tiles=((2, 2, 2), (1, 1, 1), (2, 2, 2), (2, 2, 2)), maps=(0, 0, 2, 2), deep=(N8, N8 | 1)),
    tuning(tiles=((1, 2, 3), (0, 1, 2), (3, 3, 3), (1, 1, 1)), maps=(SP | 1, 3, 1, 3), deep=(N64 | 1, N64)),
    tuning(tiles=((9, 9, 9), (9, 9, 9), (0, 3, 3), (2, 2, 4)), maps=(3, SP | 2, 0, 1), deep=(SP | N8 | 3, 2)),
    tuning(maps=(SP, SP, 0, 0), deep=(SP, 0)),
    tuning(tiles=((2, 2, 2), (1, 1, 1), (2, 2, 2), (2, 2, 2)), maps=(SP | BAL, SP | BAL | 1, BAL, BAL | 1),
           deep=(SP | BAL | N64, BAL | N64 | 1)),
    tuning(maps=(SP | BAL | 1, SP, BAL | 2, 0), deep=(SP | BAL, BAL)),
    tuning(tiles=((2, 2, 2), (1, 1, 1), (2, 2, 2), (2, 2, 2)), maps=(SP | X16, SP | X16, 2 | X16, X16),
           deep=(SP | N64 | X16, N64 | X16)),
    # slices in block order (levels 0 and 1, n >= 16), with and without XCD ranges
    tuning(tiles=((2, 2, 2), (1, 1, 1), (2, 2, 2), (2, 2, 2)), maps=(SP | CL | 1, SP | CL | X16, CL | 1, CL | 2),
           deep=(SP | N64, N64 | 1)),
    tuning(maps=(SP | CL, SP | CL | 1, CL | X16, CL | 1), deep=(SP, 0)),
]


def run(n, prec, flags, t, x, X_in=None):
    """forward of x, and inverse of X_in (default: of the forward output)"""
    plan = fcc.fcc_dct_plan_tuned(n, prec=prec, flags=flags, tuning=t)
    X = torch.empty(n ** 3, dtype=gu.cdtype(prec), device=gu.DEV)
    y = torch.empty_like(x)
    fcc.fcc_dct_forward(plan, x, X)
    fcc.fcc_dct_inverse(plan, X if X_in is None else X_in, y)
    torch.cuda.synchronize()
    out = X.cpu().numpy(), y.cpu().numpy(), fcc.fcc_dct_get_tuning(plan)
    fcc.fcc_dct_destroy(plan)
    return out


def split_key(t, n, d=0):
    """direction d's schedule parts that change which kernel evaluates an
    expression, or in which order: two-pass and balanced levels, tail depth"""
    D = n.bit_length() - 1
    lt = max(0, D - t["tail_levels"][d])
    return (tuple((bool(t["map"][d][L] & SP) or d == 1, bool(t["map"][d][L] & BAL) and (d == 1 or bool(t["map"][d][L] & SP)))
                  for L in range(lt)), t["tail_levels"][d])


@pytest.mark.parametrize("n,prec", [(4, fcc.FCC_PREC_FP64), (16, fcc.FCC_PREC_FP32), (64, fcc.FCC_PREC_FP32),
                                    (32, fcc.FCC_PREC_FP64)])
def test_tile_and_map_choices_are_bit_identical(n, prec):
    """Tiles, block numbering and node groups change no result bit; one-pass
    against two-pass levels agree to rounding."""
    x = torch.from_numpy(workloads.uniform_fp64(n, 7)).to(gu.DEV, gu.rdtype(prec))
    X0, y0, _ = run(n, prec, fcc.FCC_REAL_INPUT, SCHEDULES[0], x)
    X0_dev = torch.from_numpy(X0).to(gu.DEV)
    # a different summation order is amplified by the recursion like any other
    # rounding (about 25x per doubling of n): the FP64 parity bounds apply
    tol = {4: 1e-12, 32: 1e-10}[n] if prec == fcc.FCC_PREC_FP64 else 1e-6
    ref_by_key = {split_key(SCHEDULES[0], n): X0}
    inv_by_key = {split_key(SCHEDULES[0], n, 1): y0}
    for i, t in enumerate(SCHEDULES[1:], 1):
        X1, y1, got = run(n, prec, fcc.FCC_REAL_INPUT, t, x, X0_dev)
        key, ikey = split_key(t, n), split_key(t, n, 1)
        if key in ref_by_key:
            assert np.array_equal(ref_by_key[key].view(np.uint8), X1.view(np.uint8)), (n, i)
        ref_by_key.setdefault(key, X1)
        assert gu.maxrel(X1, X0) <= tol, (n, i)
        # every inverse reads the same X0
        if ikey in inv_by_key:
            assert np.array_equal(inv_by_key[ikey].view(np.uint8), y1.view(np.uint8)), (n, i)
        inv_by_key.setdefault(ikey, y1)
        assert gu.maxrel(y1, y0) <= tol, (n, i)
        lgm0 = max(0, n.bit_length() - 2)  # tile sides clamp to the node's cubes per side
        assert all(v <= lgm0 for v in got["tile"][0][0])


@pytest.mark.parametrize("tail", [(1, 1), (2, 3), (3, 2), (4, 4)])
def test_every_tail_depth_matches_the_oracle(tail):
    n = 16
    x = workloads.uniform_fp64(n, 11)
    ref = oracle.forward(x, n)
    xt = torch.from_numpy(x).to(gu.DEV)
    X, y, got = run(n, fcc.FCC_PREC_FP64, fcc.FCC_REAL_INPUT, tuning(tail=tail), xt)
    assert got["tail_levels"] == list(tail)
    assert gu.maxrel(X, ref) <= 1e-11
    assert gu.maxrel(y, x) <= 1e-10


@pytest.mark.parametrize("tail", [(1, 1), (3, 3), (4, 4)])
def test_tail_depth_at_n64_fp32_sampled(tail):
    n = 64
    x = workloads.gaussian_field(n, 1)
    rows = gu.sample_rows(n, 24, 3)
    ref = oracle.forward_rows(x.astype(np.float64), n, rows)
    X, y, _ = run(n, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT, tuning(tail=tail), torch.from_numpy(x).to(gu.DEV))
    assert gu.maxrel(X[rows], ref) <= 1e-5
    assert gu.maxrel(y, x) <= 1e-5


def test_autotune_choice_is_used_by_later_plans():
    n = 32
    best = fcc.fcc_dct_autotune(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT, reps=2)
    assert 1 <= best["tail_levels"][0] <= 3 and 1 <= best["tail_levels"][1] <= 3
    plan = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT)
    assert fcc.fcc_dct_get_tuning(plan) == best
    x = workloads.uniform_fp64(n, 5).astype(np.float32)
    rows = gu.sample_rows(n, 16, 4)
    X = torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV)
    fcc.fcc_dct_forward(plan, torch.from_numpy(x).to(gu.DEV), X)
    torch.cuda.synchronize()
    assert gu.maxrel(X.cpu().numpy()[rows], oracle.forward_rows(x.astype(np.float64), n, rows)) <= 1e-5
    fcc.fcc_dct_destroy(plan)


def test_batched_groups_respect_schedules():
    # two plans of the same n with different schedules in one batched call
    n = 16
    plans = [fcc.fcc_dct_plan_tuned(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT, tuning=t)
             for t in (SCHEDULES[0], tuning(tail=(3, 2), tiles=((2, 2, 2),) * 4, maps=(2, 1, 2, 1)))]
    xs = [workloads.uniform_fp64(n, 20 + i).astype(np.float32) for i in range(2)]
    ins = [torch.from_numpy(x).to(gu.DEV) for x in xs]
    outs = [torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV) for _ in xs]
    fcc.fcc_dct_batched(plans, ins, outs, 1)
    torch.cuda.synchronize()
    for x, X in zip(xs, outs):
        assert gu.maxrel(X.cpu().numpy(), oracle.forward(x.astype(np.float64), n)) <= 1e-5


@pytest.mark.parametrize("n", [8, 16, 64])
@pytest.mark.parametrize("tail", [(1, 1), (2, 1), (3, 3)])
@pytest.mark.parametrize("split", [True, False])
def test_launch_slots_match_the_bench_accounting(n, tail, split):
    """The launch slots fcc_dct_time_launches reports (including the fused
    last-level launches and the orbit-block levels) are the ones
    fcc_dct_describe_launches names and bench.py prices, in number and order:
    each slot reads and writes the method's elements once (FP32 data: real
    input 4 bytes at the top of the forward and the bottom of the inverse,
    complex 8 bytes elsewhere)."""
    maps = (SP, SP, 0, 0) if split else (0, 0, 0, 0)
    t = tuning(tail=tail, maps=maps, deep=(SP if split else 0, 0))
    for orbit in (False, True):
        if orbit:
            t["map"] = [[m | (fcc.FCC_MAP_ORBIT if (n >> L) >= 32 else 0) for L, m in enumerate(row)]
                        for row in t["map"]]
        plan = fcc.fcc_dct_plan_tuned(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT, tuning=t)
        x = torch.rand(n ** 3, device=gu.DEV)
        X = torch.empty(n ** 3, dtype=torch.complex64, device=gu.DEV)
        y = torch.empty(n ** 3, device=gu.DEV)
        for d, (src, dst) in ((1, (x, X)), (-1, (X, y))):
            ms = fcc.fcc_dct_time_launches(plan, src, dst, d, reps=1)
            slots = fcc.fcc_dct_describe_launches(plan, d)
            assert len(ms) == len(slots), (n, tail, split, d, [s["name"] for s in slots])
            assert all(v > 0 for v in ms)
            assert all(s["points"] == n ** 3 for s in slots)
            assert slots[0]["in_bytes"] == (4 if d > 0 else 8) and slots[-1]["out_bytes"] == (8 if d > 0 else 4)
            assert all(s["in_bytes"] == 8 for s in slots[1:]) and all(s["out_bytes"] == 8 for s in slots[:-1])
            assert any("orbit" in s["name"] for s in slots) == (orbit and n >= 32)
        fcc.fcc_dct_destroy(plan)
