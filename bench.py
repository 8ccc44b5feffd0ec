"""Benchmark of the fast FCC cosine transform on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c3|c4|c5] [--no-cpu] [--autotune]
                [--copy-calibration]

A step is one pass of the whole fast path over the workload's input, which is
already resident in HBM.  Default workload (c2): one forward DCT_{64x64x64} of
a smooth field (16 random Gaussians plus N(0, 0.01) noise, seed 1), FP32 data.
Other workloads:
  c1  n = 4, FP64, forward + inverse;
  c3  4096 blocks at n = 8 (8-bit levels / 255), dense split-BF16 MFMA path
      (the FP32 fast path on the same blocks is reported beside it);
  c4  n = 256 trilinear-upsampled field, FP32 data, forward + inverse, with the
      FP64 round-trip residual computed on the GPU (the variant with the top
      level in FP32 is reported beside it);
  c5  ragged batch of 512 volumes, n in {8..128}, forward + inverse in one
      graph replay, mixed precision within the workload's 1e-4: n = 8 volumes
      on split-BF16 MFMA, the top level of the others in FP32 (FP64 below);
      the split-only and the plain FP32 variants are reported beside it.
Prints ONE JSON line: points/s, the roofline of the dominant kernel (its
algorithmic bytes or flops per launch / its average duration, timed with HIP
events on the launch stream) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
MFMA_BF16_PEAK_TFS = 2500.0  # dense BF16 MFMA


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the workload, copy a 1 GiB device buffer once (the plain-copy reference for "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE scaling)")
    ap.add_argument("--autotune", action="store_true",
                    help="search the schedule before planning (setup, untimed) instead of the built-in one")
    return ap.parse_args()


def launch_bytes(n, prec, stages64, real_in, direction, sched):
    """Algorithmic bytes of each launch slot of a single-volume transform (each
    element read once and written once), in the plan's launch order."""
    N = n ** 3
    io_c = 16 if prec == 0 else 8
    io_r = 8 if prec == 0 else 4
    st = 16 if stages64 else 8
    D = n.bit_length() - 1
    SPLIT = 16
    if n == 1:
        return [("k_copy1", N * ((io_r if real_in else io_c) + io_c))]
    rin = io_r if real_in else io_c
    out = []
    if direction > 0:
        Lt = max(0, D - sched["tail_levels"][0])  # levels Lt.. run in one fused LDS launch
        # the DCT_2 pass of a two-pass level D - 2 runs with the last level
        last2 = Lt == D - 1 and D >= 3 and bool(sched["map"][0][D - 2] & SPLIT)
        for L in range(Lt):
            bi = rin if L == 0 else st
            if sched["map"][0][L] & SPLIT:
                out.append(("k_fwd_gather L%d" % L, N * (bi + st)))
                if not (last2 and L == D - 2):
                    out.append(("k_fwd_dct2 L%d" % L, N * (st + st)))
            else:
                out.append(("k_fwd_level L%d" % L, N * (bi + st)))
        if last2:
            out.append(("k_fwd_dct2_last2 L%d-%d" % (D - 2, D - 1), N * (st + io_c)))
        elif Lt == D - 1 and D >= 2:  # the last level alone: DCT_2 on the cubes
            out.append(("k_fwd_dct2 L%d" % (D - 1), N * (st + io_c)))
        else:
            out.append(("k_fwd_tail L%d-%d" % (Lt, D - 1), N * ((rin if Lt == 0 else st) + io_c)))
    else:
        Lt = max(0, D - sched["tail_levels"][1])
        # the last level and the DCT_2^-1 pass of level D - 2 run as one launch
        last2 = Lt == D - 1 and D >= 3
        if last2:
            out.append(("k_inv_dct2_last2 L%d-%d" % (D - 1, D - 2), N * (io_c + st)))
        elif Lt == D - 1 and D >= 2:  # the last level alone: DCT_2^-1 on the cubes
            out.append(("k_inv_dct2 L%d" % (D - 1), N * (io_c + st)))
        else:
            out.append(("k_inv_tail L%d-%d" % (D - 1, Lt), N * (io_c + (rin if Lt == 0 else st))))
        for L in range(Lt - 1, -1, -1):
            if not (last2 and L == D - 2):
                out.append(("k_inv_dct2 L%d" % L, N * (st + st)))
            bo = rin if L == 0 else st
            out.append(("k_inv_basis L%d" % L, N * (st + bo)))
    return out


KERNEL_SOURCES = ("paper_1807_10058_amd/csrc/fcc_dct.hip", "paper_1807_10058_amd/csrc/kernels.hpp",
                  "paper_1807_10058_amd/csrc/dense.hip", "paper_1807_10058_amd/csrc/orbits.inc")


def kernel_source_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, slot):
    """HBM bytes of one launch of `slot` from the committed rocprofv3 counter
    profile of this workload (FETCH_SIZE and WRITE_SIZE scaled by a plain copy),
    or None when there is none or the kernel sources changed since it was taken."""
    import re
    name = {"c2": "traffic_c2_n64_forward.md", "c4": "traffic_c4_n256_forward_inverse.md"}.get(workload)
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel sources sha1: ([0-9a-f]{40})", text)
    if not m or m.group(1) != kernel_source_sha1():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] == slot:
            try:
                return {"read_bytes": float(cells[2]), "write_bytes": float(cells[3]),
                        "total_bytes": float(cells[2]) + float(cells[3]), "source": "profiles/" + name}
            except ValueError:
                return None
    return None


def cpu_baseline(x, n, seconds, rng_seed=11):
    """Oracle (direct sum, 24 n^3 terms per output point) on seeded sample rows, time-bounded."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(rng_seed)
    xd = np.asarray(x, dtype=np.float64)
    done, t0 = 0, time.perf_counter()
    chunk = max(8, oracle.num_threads())
    while time.perf_counter() - t0 < seconds:
        rows = rng.choice(n ** 3, chunk, replace=False)
        oracle.forward_rows(xd, n, rows)
        done += chunk
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d of %d output points of one n=%d forward, direct 24*n^3-term sum each, %.1f s"
                      % (done, n ** 3, n, dt)}


def time_steps(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, time.perf_counter() - wall0


def single_volume(args, name):
    """c1, c2, c4: one volume per step."""
    import numpy as np
    import torch

    import oracle
    import paper_1807_10058_amd as fcc
    import workloads
    from tests.gpu_util import sample_rows
    if name == "c1":
        n, x_np, prec, direction = 4, workloads.uniform_fp64(4, 0), fcc.FCC_PREC_FP64, 0
        desc = "c1: single FCC-DCT forward+inverse, n=4, uniform[-1,1] FP64, seed 0"
    elif name == "c2":
        n, x_np, prec, direction = 64, workloads.gaussian_field(64, 1), fcc.FCC_PREC_FP32, 1
        desc = "c2: single FCC-DCT forward, n=64, 16 Gaussians + N(0,0.01) noise, FP32 data, seed 1"
    else:
        n, x_np, prec, direction = 256, workloads.upsampled_field(256, 3), fcc.FCC_PREC_FP32, 0
        desc = "c4: single FCC-DCT forward+inverse, n=256, trilinear-upsampled 16^3 uniform[-1,1], FP32 data, seed 3"
    dev = torch.device("cuda:0")
    rdt = torch.float64 if prec == fcc.FCC_PREC_FP64 else torch.float32
    cdt = torch.complex128 if prec == fcc.FCC_PREC_FP64 else torch.complex64
    t0 = time.perf_counter()
    if args.autotune:
        fcc.fcc_dct_autotune(n, prec=prec, flags=fcc.FCC_REAL_INPUT, reps=5)
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = fcc.fcc_dct_plan(n, prec=prec, flags=fcc.FCC_REAL_INPUT)
    plan_s = time.perf_counter() - t0
    sched = fcc.fcc_dct_get_tuning(plan)
    stages64 = prec == fcc.FCC_PREC_FP64 or n > 4
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(dev, rdt)
    X = torch.empty(n ** 3, dtype=cdt, device=dev)
    y = torch.empty(n ** 3, dtype=rdt, device=dev)

    def step():
        fcc.fcc_dct_forward(plan, x, X)
        if direction == 0:
            fcc.fcc_dct_inverse(plan, X, y)

    ms, wall = time_steps(step, args.steps, args.warmup)
    points = n ** 3
    slots = []
    direction_ms = {}
    for d in ([1] if direction == 1 else [1, -1]):
        src, dst = (x, X) if d == 1 else (X, y)
        times = fcc.fcc_dct_time_launches(plan, src, dst, d, reps=max(5, min(args.steps, 50)))
        direction_ms["forward" if d == 1 else "inverse"] = round(float(sum(times)), 5)
        for (kname, nbytes), t in zip(launch_bytes(n, prec, stages64, True, d, sched), times):
            slots.append((kname, nbytes, t))
    kname, nbytes, tdom = max(slots, key=lambda s: s[2])
    achieved = nbytes / (tdom * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name, kname), "launch_ms": tdom,
            "algorithmic_bytes": nbytes}
    step()
    torch.cuda.synchronize()
    rows = sample_rows(n, 48, 5)
    Xh = X.cpu().numpy().astype(np.complex128)
    ref = oracle.forward_rows(np.asarray(x_np, dtype=np.float64), n, rows)
    acc = {"forward_max_rel_sampled": float(np.abs(Xh[rows] - ref).max() / np.abs(ref).max()),
           "rows": int(len(rows))}
    if direction == 0:
        acc["roundtrip_max_rel_fp64_gpu"] = fcc.fcc_dct_roundtrip_residual(plan, x, y)
    cfg = {"workload": desc, "n": n, "points": points, "io_dtype": "f64" if prec == 0 else "f32",
           "stages": "f64" if stages64 else "f32", "direction": "forward" if direction == 1 else "forward+inverse",
           "plan_seconds": round(plan_s, 3), "autotune_seconds": round(tune_s, 3), "schedule": sched,
           "wall_seconds_timed": round(wall, 4)}
    # kernel time of each direction (sum of its launches, HIP events)
    extra = {"launches_ms": {s[0]: round(s[2], 5) for s in slots}, "direction_kernel_ms": direction_ms,
             "accuracy": acc}
    if name == "c4":
        # beside the line: the top level in FP32 (FP64 below), same input
        p32 = fcc.fcc_dct_plan(n, prec=prec, flags=fcc.FCC_REAL_INPUT | fcc.FCC_LEVEL0_FP32)

        def step32():
            fcc.fcc_dct_forward(p32, x, X)
            fcc.fcc_dct_inverse(p32, X, y)

        ms32, _ = time_steps(step32, args.steps, args.warmup)
        step32()
        torch.cuda.synchronize()
        X32 = X.cpu().numpy().astype(np.complex128)
        extra["variants"] = {"level0_fp32": {
            "ms_per_step": ms32, "points_per_s": points / (ms32 * 1e-3),
            "accuracy": {"forward_max_rel_sampled": float(np.abs(X32[rows] - ref).max() / np.abs(ref).max()),
                         "roundtrip_max_rel_fp64_gpu": fcc.fcc_dct_roundtrip_residual(p32, x, y)}}}
        fcc.fcc_dct_destroy(p32)
    return points, ms, "f64" if stages64 else "f32", cfg, roof, extra, (x_np, n)


def batched(args, name):
    """c3, c5: many volumes per step through fcc_dct_batched (one graph replay)."""
    import numpy as np
    import torch

    import oracle
    import paper_1807_10058_amd as fcc
    import workloads
    from tests.gpu_util import sample_rows
    dev = torch.device("cuda:0")
    if name == "c3":
        blocks = workloads.quantised_blocks(4096, 8, seed=2)
        ns = [8] * blocks.shape[0]
        xs_np = list(blocks)
        direction = 1
        desc = "c3: 4096 independent FCC-DCT blocks at n=8, 8-bit levels/255 FP32 (seed 2), forward"
    else:
        ns, xs_np = workloads.ragged_batch(512, seed=4)
        direction = 0
        desc = ("c5: ragged batch of 512 FCC-DCT volumes, n from {8,16,32,64,128} (seed 4), N(0,1) FP32, "
                "forward then inverse in one graph replay")
    points = int(sum(n ** 3 for n in ns))
    cache = {}
    t0 = time.perf_counter()
    if args.autotune:
        for n in sorted(set(ns)):
            if n > 1:
                fcc.fcc_dct_autotune(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT, reps=3)
    tune_s = time.perf_counter() - t0

    def plan_for(n, prec):
        if (n, prec) not in cache:
            cache[(n, prec)] = fcc.fcc_dct_plan(n, prec=prec, flags=fcc.FCC_REAL_INPUT)
        return cache[(n, prec)]

    if name == "c3":
        flat = torch.from_numpy(np.ascontiguousarray(blocks)).to(dev)
        xs = [flat[b] for b in range(len(ns))]
    else:
        xs = [torch.from_numpy(x).to(dev) for x in xs_np]
    outs = [torch.empty(n ** 3, dtype=torch.complex64, device=dev) for n in ns]

    def plan_for_variant(n, variant):
        # split: split-BF16 dense path for n <= 8; mixed: that, and the top level
        # in FP32 for larger n (round trip ~4e-6, within the 1e-4 of this workload)
        if variant in ("split", "mixed") and n <= 8:
            return plan_for(n, fcc.FCC_PREC_SPLIT_BF16)
        if variant == "mixed":
            key = (n, "level0_fp32")
            if key not in cache:
                cache[key] = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32,
                                              flags=fcc.FCC_REAL_INPUT | fcc.FCC_LEVEL0_FP32)
            return cache[key]
        return plan_for(n, fcc.FCC_PREC_FP32)

    def run(variant):
        plans = [plan_for_variant(n, variant) for n in ns]
        step = fcc.BatchedCall(plans, xs, outs, direction)
        t0 = time.perf_counter()
        step()  # records the graph
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        ms, wall = time_steps(step, args.steps, args.warmup)
        return plans, step, ms, wall, build_s

    originals = [x.clone() for x in xs] if direction == 0 else None
    res = {}
    variants = ("split", "fp32") if name == "c3" else ("mixed", "split", "fp32")
    for variant in variants:
        if direction == 0:
            for x, o in zip(xs, originals):
                x.copy_(o)
        plans, step, ms, wall, build_s = run(variant)
        # accuracy: forward outputs vs oracle (sampled), round trip vs input
        if direction == 0:
            for x, o in zip(xs, originals):
                x.copy_(o)
        step()
        torch.cuda.synchronize()
        worst_f, worst_rt = 0.0, 0.0
        check = list(range(0, len(ns), max(1, len(ns) // 24)))
        for i in check:
            n = ns[i]
            rows = sample_rows(n, 16, i)
            ref = oracle.forward_rows(np.asarray(xs_np[i], dtype=np.float64), n, rows)
            got = outs[i].cpu().numpy().astype(np.complex128)[rows]
            worst_f = max(worst_f, float(np.abs(got - ref).max() / np.abs(ref).max()))
            if direction == 0:
                worst_rt = max(worst_rt, float((xs[i].cpu().double() - originals[i].cpu().double()).abs().max()
                                               / originals[i].abs().max().item()))
        acc = {"forward_max_rel_sampled": worst_f, "volumes_checked": len(check)}
        if direction == 0:
            acc["roundtrip_max_rel"] = worst_rt
        res[variant] = {"ms_per_step": ms, "points_per_s": points / (ms * 1e-3), "accuracy": acc,
                        "graph_build_s": round(build_s, 3), "wall_seconds_timed": round(wall, 4)}
    main = res["split"] if name == "c3" else res["mixed"]
    if name == "c3":
        # one GEMM launch per step: out[4096 x 1024] = in[4096 x 512] W^T, 3 split products
        flops = 2.0 * 4096 * 1024 * 512 * 3
        achieved = flops / (main["ms_per_step"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "k_split_gemm<bf16>", "achieved": achieved,
                "peak": MFMA_BF16_PEAK_TFS, "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFS,
                "traffic": None, "launch_ms": main["ms_per_step"], "algorithmic_flops": flops}
        dtype = "bf16x3 (split) / f32 acc"
    else:
        # dominant kernels are the fast-path levels of the n = 128 volumes; report the whole-step
        # algorithmic bytes (FP32 in 4 + complex64 out 8, then back) over the step time
        nbytes = points * (4 + 8 + 8 + 4)
        achieved = nbytes / (main["ms_per_step"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "whole step (graph replay)", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "launch_ms": main["ms_per_step"], "algorithmic_bytes": nbytes}
        dtype = "f64 stages, f32 top level (n >= 16); bf16x3 split (n = 8)"
    cfg = {"workload": desc, "volumes": len(ns), "points": points, "io_dtype": "f32",
           "sizes": {str(k): ns.count(k) for k in sorted(set(ns))}, "autotune_seconds": round(tune_s, 3)}
    extra = {"variants": res, "accuracy": main["accuracy"]}
    big = max(range(len(ns)), key=lambda i: ns[i])
    return points, main["ms_per_step"], dtype, cfg, roof, extra, (xs_np[big], ns[big])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("c1", "c2", "c4"):
        points, ms, dtype, cfg, roof, extra, cpu_case = single_volume(args, args.workload)
    else:
        points, ms, dtype, cfg, roof, extra, cpu_case = batched(args, args.workload)
    out = {
        "metric": "FCC-DCT points/s", "value": points / (ms * 1e-3), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg,
        "roofline": roof,
    }
    out.update(extra)
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        b = a.clone()
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = int(b.numel() * 4)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cpu_case[0], cpu_case[1], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
