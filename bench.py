"""Benchmark of the fast FCC cosine transform on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c4|c1] [--no-cpu]

A step is one pass of the whole fast path over the workload's input, already
resident in HBM.  Default workload (c2): one forward DCT_{64x64x64} of a
smooth field (16 random Gaussians plus N(0, 0.01) noise, seed 1), FP32 data.
Prints ONE JSON line with points/s, the roofline of the dominant kernel
(algorithmic bytes of that launch / its average duration, timed with HIP
events on the launch stream) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def workload(name):
    import numpy as np

    import workloads
    import paper_1807_10058_amd as fcc
    if name == "c1":
        return dict(n=4, x=workloads.uniform_fp64(4, 0), prec=fcc.FCC_PREC_FP64, direction=0,
                    desc="c1: single FCC-DCT forward+inverse, n=4, uniform[-1,1] FP64, seed 0")
    if name == "c2":
        return dict(n=64, x=workloads.gaussian_field(64, 1), prec=fcc.FCC_PREC_FP32, direction=1,
                    desc="c2: single FCC-DCT forward, n=64, 16 Gaussians + N(0,0.01) noise, FP32 data, seed 1")
    if name == "c4":
        return dict(n=256, x=workloads.upsampled_field(256, 3), prec=fcc.FCC_PREC_FP32, direction=0,
                    desc="c4: single FCC-DCT forward+inverse, n=256, trilinear-upsampled 16^3 noise, FP32, seed 3")
    raise ValueError(name)


def launch_bytes(n, prec, stages64, real_in, direction):
    """Algorithmic bytes of each launch slot (each element read once, written once)."""
    N = n ** 3
    io_c = 16 if prec == 0 else 8
    io_r = 8 if prec == 0 else 4
    st = 16 if stages64 else 8
    D = n.bit_length() - 1
    out = []
    if direction > 0:
        for L in range(D):
            bi = (io_r if real_in else io_c) if L == 0 else st
            bo = io_c if L == D - 1 else st
            out.append(("fwd_level%d" % L, N * (bi + bo)))
    else:
        for k, L in enumerate(range(D - 1, -1, -1)):
            bi = io_c if k == 0 else st
            out.append(("inv_dct2_level%d" % L, N * (bi + st)))
            bo = (io_r if real_in else io_c) if L == 0 else st
            out.append(("inv_basis_level%d" % L, N * (st + bo)))
    return out


def cpu_baseline(x, n, seconds, rng_seed=11):
    """Oracle (direct O(N) per output point) on seeded sample rows, time-bounded."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(rng_seed)
    xd = x.astype(np.float64)
    done, t0 = 0, time.perf_counter()
    chunk = max(8, oracle.num_threads())
    while time.perf_counter() - t0 < seconds:
        rows = rng.choice(n ** 3, chunk, replace=False)
        oracle.forward_rows(xd, n, rows)
        done += chunk
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d of %d output points of the n=%d forward, direct 24*N-term sum each, %.1f s"
                      % (done, n ** 3, n, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1807_10058_amd as fcc
    w = workload(args.workload)
    n, prec, direction = w["n"], w["prec"], w["direction"]
    dev = torch.device("cuda:0")
    rdt = torch.float64 if prec == fcc.FCC_PREC_FP64 else torch.float32
    cdt = torch.complex128 if prec == fcc.FCC_PREC_FP64 else torch.complex64
    t0 = time.perf_counter()
    plan = fcc.fcc_dct_plan(n, prec=prec, flags=fcc.FCC_REAL_INPUT)
    plan_s = time.perf_counter() - t0
    stages64 = prec == fcc.FCC_PREC_FP64 or n > 8
    x = torch.from_numpy(np.ascontiguousarray(w["x"])).to(dev, rdt)
    X = torch.empty(n ** 3, dtype=cdt, device=dev)
    y = torch.empty(n ** 3, dtype=rdt, device=dev)

    def step():
        fcc.fcc_dct_forward(plan, x, X)
        if direction == 0:
            fcc.fcc_dct_inverse(plan, X, y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    points = n ** 3
    value = points / (ms * 1e-3)

    # roofline of the dominant kernel: per-launch HIP events on the launch stream
    slots = []
    for d in ([1] if direction == 1 else [1, -1]):
        src, dst = (x, X) if d == 1 else (X, y)
        times = fcc.fcc_dct_time_launches(plan, src, dst, d, reps=max(5, min(args.steps, 50)))
        for (name, nbytes), t in zip(launch_bytes(n, prec, stages64, True, d), times):
            slots.append((name, nbytes, t))
    name, nbytes, tdom = max(slots, key=lambda s: s[2])
    achieved = nbytes / (tdom * 1e-3) / 1e9

    # accuracy of this run on sampled outputs (oracle, FP64)
    import oracle
    from tests.gpu_util import sample_rows
    rows = sample_rows(n, 48, 5)
    step()
    torch.cuda.synchronize()
    Xh = X.cpu().numpy().astype(np.complex128)
    ref = oracle.forward_rows(w["x"].astype(np.float64), n, rows)
    err = float(np.abs(Xh[rows] - ref).max() / np.abs(ref).max())
    acc = {"forward_max_rel_sampled": err, "rows": int(len(rows))}
    if direction == 0:
        acc["roundtrip_max_rel"] = float((y.cpu().double() - torch.from_numpy(w["x"]).double()).abs().max()
                                         / abs(w["x"]).max())

    out = {
        "metric": "FCC-DCT points/s", "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if stages64 else "f32", "data": "synthetic",
        "config": {"workload": w["desc"], "n": n, "points": points, "io_dtype": "f64" if prec == 0 else "f32",
                   "stages": "f64" if stages64 else "f32", "direction": "forward" if direction == 1 else "forward+inverse",
                   "plan_seconds": round(plan_s, 3), "wall_seconds_timed": round(wall, 4)},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "launch_ms": tdom,
                     "algorithmic_bytes": nbytes},
        "launches_ms": {s[0]: round(s[2], 5) for s in slots},
        "accuracy": acc,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w["x"], n, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
