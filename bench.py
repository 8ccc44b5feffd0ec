"""Benchmark of the fast FCC cosine transform on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|c1|c2|c3|c4] [--no-cpu] [--autotune]
                [--copy-calibration] [--pmc-pass] [--summarize DIR]

A step is one pass of the whole fast path over the workload's input, which is
already resident in HBM.  Default workload (c5): the ragged batch of 512
volumes, n drawn from {8, 16, 32, 64, 128} (seed 4), N(0,1) FP32 data,
forward then inverse in one replay of the recorded HIP graph.  Its line is the
hybrid mixed-precision variant (n = 8 volumes on the split-BF16 MFMA path; the
others with the top level in FP32 arithmetic, FP64 stages below and the
forward's last levels as one dense base per node of size min(16, n / 2),
FCC_FOLD_BASE); the same without the dense base, the split-only and the plain
variant (FP32 data, FP64 stages) are reported beside it, with the n = 256
single-volume forward + inverse (c4).
Other workloads:
  c1  n = 4, FP64, forward + inverse;
  c2  n = 64 forward of a smooth field, FP32 data;
  c3  4096 blocks at n = 8 (8-bit levels / 255), dense split-BF16 MFMA path
      (the FP32 fast path on the same blocks is reported beside it);
  c4  n = 256 trilinear-upsampled field, FP32 data, forward + inverse (dense
      base of node size 16 in the forward), with the FP64 round-trip residual
      computed on the GPU.
Prints ONE JSON line: points/s, the roofline of the dominant kernel (the
launch slot with the longest average duration, timed with start/stop events
recorded by each launch on its own stream; its algorithmic bytes = the
method's input and output of that launch, each element once, in the data
precision) and the CPU oracle timed on a bounded sample.

--pmc-pass runs only the workload's launch slots once, eagerly, in slot order
(for rocprofv3 counter runs) and writes their list to gpurun_out/slots_<w>.json;
--summarize DIR turns a counter run's CSV output in DIR into the traffic table
of profiles/traffic_<w>.md; with --fold both cover the fold+FFT variant's
launches (c4, c5), which the c5 line reports beside the paper's factorisation.
"""
import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
MFMA_BF16_PEAK_TFS = 2500.0  # dense BF16 MFMA
KERNEL_SOURCES = ("paper_1807_10058_amd/csrc/fcc_dct.hip", "paper_1807_10058_amd/csrc/kernels.hpp",
                  "paper_1807_10058_amd/csrc/orbit_level.hpp", "paper_1807_10058_amd/csrc/dense.hip",
                  "paper_1807_10058_amd/csrc/orbits.inc", "paper_1807_10058_amd/csrc/fold_fft.hpp",
                  "paper_1807_10058_amd/csrc/base_fold.hpp")
TRAFFIC_PROFILE = {"c2": "traffic_c2_n64_forward.md", "c4": "traffic_c4_n256_forward_inverse.md",
                   "c5": "traffic_c5_ragged512_forward_inverse.md",
                   "c4_fold": "traffic_fold_c4_n256_forward_inverse.md",
                   "c5_fold": "traffic_fold_c5_ragged512_forward_inverse.md"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-c4", action="store_true", help="c5: skip the n = 256 single-volume report beside the line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the workload, copy a 1 GiB device buffer once (the plain-copy reference for "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE scaling)")
    ap.add_argument("--autotune", action="store_true",
                    help="search the schedule before planning (setup, untimed) instead of the built-in one")
    ap.add_argument("--pmc-pass", action="store_true", help="one eager pass of the launch slots only")
    ap.add_argument("--summarize", metavar="DIR", help="write the traffic table of a counter run in DIR")
    ap.add_argument("--fold", action="store_true",
                    help="with --pmc-pass / --summarize: the launches of the fold+FFT variant (c4, c5)")
    return ap.parse_args()


def kernel_source_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, slot):
    """HBM bytes of one launch of `slot` (mean over the slots of that name) from
    the committed rocprofv3 counter table of this workload, or None when there
    is none or the kernel sources changed since it was taken."""
    import re
    name = TRAFFIC_PROFILE.get(workload)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel sources sha1: ([0-9a-f]{40})", text)
    if not m or m.group(1) != kernel_source_sha1():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == slot:
            try:
                rd, wr = float(cells[2]), float(cells[3])
            except ValueError:
                return None
            return {"read_bytes": rd, "write_bytes": wr, "total_bytes": rd + wr, "source": "profiles/" + name}
    return None


def roofline(workload, slots):
    """Roofline entry of the dominant (slowest) launch slot."""
    dom = max(slots, key=lambda s: s["ms"])
    nbytes = dom["points"] * (dom["in_bytes"] + dom["out_bytes"])
    achieved = nbytes / (dom["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(workload, dom["name"]),
            "launch_ms": dom["ms"], "algorithmic_bytes": nbytes}


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
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, time.perf_counter() - wall0


def single_slots(plan, pairs, reps):
    """Timed launch slots of a single-volume plan: [(direction, src, dst)]."""
    import paper_1807_10058_amd as fcc
    out = []
    for d, src, dst in pairs:
        info = fcc.fcc_dct_describe_launches(plan, d)
        times = fcc.fcc_dct_time_launches(plan, src, dst, d, reps=reps)
        for i, t in zip(info, times):
            out.append(dict(i, ms=float(t), direction="forward" if d > 0 else "inverse"))
    return out


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
    fold = args.fold and args.pmc_pass and name == "c4"
    flags = fcc.FCC_REAL_INPUT | (fcc.FCC_FOLD_FFT if fold else (fcc.FCC_FOLD_BASE if name == "c4" else 0))
    plan = fcc.fcc_dct_plan(n, prec=prec, flags=flags)
    plan_s = time.perf_counter() - t0
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(dev, rdt)
    X = torch.empty(n ** 3, dtype=cdt, device=dev)
    y = torch.empty(n ** 3, dtype=rdt, device=dev)
    pairs = [(1, x, X)] + ([(-1, X, y)] if direction == 0 else [])
    if args.pmc_pass:
        return pmc_pass(name + ("_fold" if fold else ""), lambda: single_slots(plan, pairs, 1))

    def step():
        fcc.fcc_dct_forward(plan, x, X)
        if direction == 0:
            fcc.fcc_dct_inverse(plan, X, y)

    ms, wall = time_steps(step, args.steps, args.warmup)
    slots = single_slots(plan, pairs, max(5, min(args.steps, 50)))
    roof = roofline(name, slots)
    step()
    torch.cuda.synchronize()
    rows = sample_rows(n, 48, 5)
    Xh = X.cpu().numpy().astype(np.complex128)
    ref = oracle.forward_rows(np.asarray(x_np, dtype=np.float64), n, rows)
    acc = {"forward_max_rel_sampled": float(np.abs(Xh[rows] - ref).max() / np.abs(ref).max()),
           "rows": int(len(rows))}
    if direction == 0:
        acc["roundtrip_max_rel_fp64_gpu"] = fcc.fcc_dct_roundtrip_residual(plan, x, y)
    cfg = {"workload": desc, "n": n, "points": n ** 3, "io_dtype": "f64" if prec == 0 else "f32",
           "direction": "forward" if direction == 1 else "forward+inverse",
           "plan_seconds": round(plan_s, 3), "autotune_seconds": round(tune_s, 3),
           "schedule": fcc.fcc_dct_get_tuning(plan), "wall_seconds_timed": round(wall, 4)}
    dirs = {}
    for s in slots:
        dirs[s["direction"]] = round(dirs.get(s["direction"], 0.0) + s["ms"], 5)
    extra = {"launches_ms": {s["name"]: round(s["ms"], 5) for s in slots}, "direction_kernel_ms": dirs,
             "accuracy": acc}
    dtype = "f64" if prec == fcc.FCC_PREC_FP64 else "f32 data, f64 stages"
    return n ** 3, ms, dtype, cfg, roof, extra, (x_np, n)


def pmc_pass(name, run_slots):
    """One eager pass of the launch slots (for counter runs); writes their list."""
    import torch
    slots = run_slots()
    torch.cuda.synchronize()
    os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
    path = os.path.join(ROOT, "gpurun_out", "slots_%s.json" % name)
    with open(path, "w") as f:
        json.dump([{k: s[k] for k in ("name", "points", "in_bytes", "out_bytes")} for s in slots], f)
    print(json.dumps({"pmc_pass": name, "slots": len(slots), "list": path}), flush=True)
    return None


def c4_beside(args):
    """The n = 256 single-volume forward + inverse, reported beside the c5 line."""
    import numpy as np
    import torch

    import oracle
    import paper_1807_10058_amd as fcc
    import workloads
    from tests.gpu_util import sample_rows
    n = 256
    dev = torch.device("cuda:0")
    x_np = workloads.upsampled_field(n, 3)
    plan = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_BASE)
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(dev)
    X = torch.empty(n ** 3, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)

    def step():
        fcc.fcc_dct_forward(plan, x, X)
        fcc.fcc_dct_inverse(plan, X, y)

    ms, _ = time_steps(step, max(5, args.steps // 2), 2)
    # the radix-2 levels all the way down (no dense base), same input
    rplan = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT)

    def rstep():
        fcc.fcc_dct_forward(rplan, x, X)
        fcc.fcc_dct_inverse(rplan, X, y)

    rms, _ = time_steps(rstep, max(5, args.steps // 2), 2)
    rdirs = {}
    for s_ in single_slots(rplan, [(1, x, X), (-1, X, y)], 10):
        rdirs[s_["direction"]] = round(rdirs.get(s_["direction"], 0.0) + s_["ms"], 5)
    slots = single_slots(plan, [(1, x, X), (-1, X, y)], 10)
    roof = roofline("c4", slots)
    dirs = {}
    for s in slots:
        dirs[s["direction"]] = round(dirs.get(s["direction"], 0.0) + s["ms"], 5)
    step()
    torch.cuda.synchronize()
    out = {"workload": "c4: n=256 forward+inverse, trilinear-upsampled field, FP32 data, FP64 stages, "
                       "forward with the dense base of node size 16",
           "ms_per_step": ms, "points_per_s": n ** 3 / (ms * 1e-3), "direction_kernel_ms": dirs,
           "radix2_to_the_end": {"ms_per_step": rms, "direction_kernel_ms": rdirs},
           "roofline": roof, "roundtrip_max_rel_fp64_gpu": fcc.fcc_dct_roundtrip_residual(plan, x, y),
           "step_frac_of_hbm_floor": (n ** 3 * 28) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    # the fold+FFT variant on the same input (FP32 arithmetic throughout)
    fplan = fcc.fcc_dct_plan(n, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_FFT)

    def fstep():
        fcc.fcc_dct_forward(fplan, x, X)
        fcc.fcc_dct_inverse(fplan, X, y)

    fms, _ = time_steps(fstep, max(5, args.steps // 2), 2)
    fslots = single_slots(fplan, [(1, x, X), (-1, X, y)], 10)
    fdirs = {}
    for s in fslots:
        fdirs[s["direction"]] = round(fdirs.get(s["direction"], 0.0) + s["ms"], 5)
    fstep()
    torch.cuda.synchronize()
    rows = sample_rows(n, 16, 3)
    ref = oracle.forward_rows(np.asarray(x_np, dtype=np.float64), n, rows)
    got = X.cpu().numpy().astype(np.complex128)[rows]
    out["fold_fft_variant"] = {
        "what": "fold+FFT formulation (from the explicit matrix; not the paper's factorisation), FP32 arithmetic",
        "ms_per_step": fms, "points_per_s": n ** 3 / (fms * 1e-3), "direction_kernel_ms": fdirs,
        "roofline": roofline("c4_fold", fslots), "forward_max_rel_sampled": float(np.abs(got - ref).max()
                                                                               / np.abs(ref).max()),
        "roundtrip_max_rel_fp64_gpu": fcc.fcc_dct_roundtrip_residual(fplan, x, y),
        "step_frac_of_hbm_floor": (n ** 3 * 28) / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


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

    def plan_for(n, prec, flags=fcc.FCC_REAL_INPUT):
        if (n, prec, flags) not in cache:
            cache[(n, prec, flags)] = fcc.fcc_dct_plan(n, prec=prec, flags=flags)
        return cache[(n, prec, flags)]

    if name == "c3":
        flat = torch.from_numpy(np.ascontiguousarray(blocks)).to(dev)
        xs = [flat[b] for b in range(len(ns))]
    else:
        xs = [torch.from_numpy(x).to(dev) for x in xs_np]
    outs = [torch.empty(n ** 3, dtype=torch.complex64, device=dev) for n in ns]

    def plan_for_variant(n, variant):
        # split: the split-BF16 dense MFMA path for n <= 8; mixed: that, and the
        # top level in FP32 arithmetic for larger n (FP64 stages below);
        # hybrid: mixed with the forward's dense base per node
        if variant in ("split", "mixed", "hybrid") and n <= 8:
            return plan_for(n, fcc.FCC_PREC_SPLIT_BF16)
        if variant == "mixed":
            return plan_for(n, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_LEVEL0_FP32)
        if variant == "hybrid":
            return plan_for(n, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_LEVEL0_FP32 | fcc.FCC_FOLD_BASE)
        if variant == "fold":
            return plan_for(n, fcc.FCC_PREC_FP32, fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_FFT)
        return plan_for(n, fcc.FCC_PREC_FP32)

    main_variant = "split" if name == "c3" else "hybrid"
    if args.pmc_pass:
        fold = args.fold and name == "c5"
        plans = [plan_for_variant(n, "fold" if fold else main_variant) for n in ns]
        return pmc_pass(name + ("_fold" if fold else ""),
                        lambda: fcc.fcc_dct_batched_time_launches(plans, xs, outs, direction, reps=1))

    originals = [x.clone() for x in xs] if direction == 0 else None
    res = {}
    slots_main = None
    variants = ("split", "fp32") if name == "c3" else ("hybrid", "mixed", "split", "fp32", "fold")
    for variant in variants:
        if direction == 0:
            for x, o in zip(xs, originals):
                x.copy_(o)
        plans = [plan_for_variant(n, variant) for n in ns]
        step = fcc.BatchedCall(plans, xs, outs, direction)
        t0 = time.perf_counter()
        step()  # records the graph
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        ms, wall = time_steps(step, args.steps, args.warmup)
        if variant == main_variant:
            slots_main = fcc.fcc_dct_batched_time_launches(plans, xs, outs, direction, reps=3)
        if variant == "fold":
            slots_fold = fcc.fcc_dct_batched_time_launches(plans, xs, outs, direction, reps=3)
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
        if variant == "fold":
            res[variant]["roofline"] = roofline(name + "_fold", slots_fold)
        fcc.fcc_dct_batched_release()
    main = res[main_variant]
    if name == "c3":
        # per step: the split of the input into hi + lo, then one GEMM launch
        # out[4096 x 1024] = in[4096 x 512] W^T with 3 split products (the roofline's kernel)
        flops = 2.0 * 4096 * 1024 * 512 * 3
        gemm = [sl for sl in slots_main if "k_split_gemm" in sl["name"]][0]
        t = gemm["ms"]
        achieved = flops / (t * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": gemm["name"], "achieved": achieved,
                "peak": MFMA_BF16_PEAK_TFS, "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFS,
                "traffic": None, "launch_ms": t, "algorithmic_flops": flops}
        dtype = "bf16x3 (split) / f32 acc"
    else:
        roof = roofline(name, slots_main)
        dtype = "mixed: f32 top level + f64 stages and base (n >= 16), bf16x3 split MFMA (n = 8); f32 data"
    cfg = {"workload": desc, "volumes": len(ns), "points": points, "io_dtype": "f32",
           "sizes": {str(k): ns.count(k) for k in sorted(set(ns))}, "autotune_seconds": round(tune_s, 3),
           "variants": {"hybrid": "split-BF16 MFMA for n = 8; FP32 top level, FP64 stages below and the "
                                  "forward's dense base of node size min(16, n/2) for n >= 16",
                        "mixed": "split-BF16 MFMA for n = 8; FP32 top level, FP64 stages below for n >= 16",
                        "split": "split-BF16 MFMA for n = 8; FP64 stages for n >= 16",
                        "fp32": "FP32 data, FP64 stages for every n (plain fast path)",
                        "fold": "fold+FFT formulation from the explicit matrix (a variant, not the paper's "
                                "factorisation), FP32 arithmetic throughout"}}
    slot_ms = {}
    for s in slots_main:
        slot_ms[s["name"]] = round(slot_ms.get(s["name"], 0.0) + s["ms"], 5)
    extra = {"variants": res, "accuracy": main["accuracy"], "slot_ms_sum": round(sum(slot_ms.values()), 4),
             "launches_ms": slot_ms}
    if name == "c5" and not args.no_c4:
        extra["c4_beside"] = c4_beside(args)
    big = max(range(len(ns)), key=lambda i: ns[i])
    return points, main["ms_per_step"], dtype, cfg, roof, extra, (xs_np[big], ns[big])


def _fcc_dispatches(rows):
    """(dispatch id, kernel name) of the transform's own kernels, in dispatch order."""
    out = [(d, kn) for d, kn in rows if "fcc::k_" in kn]
    return [r for r in out if "k_phase_table" not in r[1] and "k_node_table" not in r[1]]


def summarize(directory, workload):
    """Per-slot tables of a --pmc-pass run under rocprofv3 (the last len(slots)
    transform dispatches are the slots, in order): from a kernel trace
    (DIR/prof_<w>: durations) or from a FETCH_SIZE and a WRITE_SIZE counter
    run (DIR/pmc_<w>_FETCH_SIZE, DIR/pmc_<w>_WRITE_SIZE, each ending with the
    1 GiB calibration copy of --copy-calibration)."""
    import csv
    slots = json.load(open(os.path.join(ROOT, "gpurun_out", "slots_%s.json" % workload)))
    print("kernel sources sha1: %s" % kernel_source_sha1())
    trace = glob.glob(os.path.join(directory, "prof_%s" % workload, "**", "*kernel_trace.csv"), recursive=True)
    if trace:
        rows = []
        for r in csv.DictReader(open(trace[0])):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        rows.sort()
        dur = {d: t for d, _, t in rows}
        last = _fcc_dispatches([(d, kn) for d, kn, _ in rows])[-len(slots):]
        agg = {}
        for sl, (d, kn) in zip(slots, last):
            a = agg.setdefault(sl["name"], {"kernel": kn, "k": 0, "ns": 0.0, "alg": 0.0})
            a["k"] += 1
            a["ns"] += dur[d]
            a["alg"] += sl["points"] * (sl["in_bytes"] + sl["out_bytes"])
        print("| Slot | Kernel | Launches | Trace mean (us) | Algorithmic GB/s |")
        print("|:--|:--|--:|--:|--:|")
        for nm, a in agg.items():
            print("| %s | %s | %d | %.2f | %.0f |" % (nm, a["kernel"].replace("void fcc::", "").split("(")[0], a["k"],
                                                     a["ns"] / a["k"] / 1e3, a["alg"] / a["ns"]))
    if not glob.glob(os.path.join(directory, "pmc_%s_FETCH_SIZE" % workload)):
        return
    vals = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        files = glob.glob(os.path.join(directory, "pmc_%s_%s" % (workload, counter), "**", "*counter_collection.csv"),
                          recursive=True)
        if not files:
            raise SystemExit("no counter_collection.csv for %s under %s" % (counter, directory))
        per, names = {}, {}
        for r in csv.DictReader(open(files[0])):
            d = int(r["Dispatch_Id"])
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
        order = sorted(per)
        copies = [d for d in order if "copyBuffer" in names[d]]
        calib = per[copies[-1]] if copies else None
        last = _fcc_dispatches([(d, names[d]) for d in order])[-len(slots):]
        vals[counter] = ([per[d] for d, _ in last], [kn for _, kn in last], calib)
    fetch, names, cal_f = vals["FETCH_SIZE"]
    write, _, cal_w = vals["WRITE_SIZE"]
    gib_kib = 1 << 20
    f_scale = gib_kib / cal_f if cal_f else 2.0
    w_scale = gib_kib / cal_w if cal_w else 1.0
    agg = {}
    for sl, kn, f, w in zip(slots, names, fetch, write):
        a = agg.setdefault(sl["name"], {"kernel": kn, "k": 0, "f": 0.0, "w": 0.0, "alg": 0.0})
        a["k"] += 1
        a["f"] += f * f_scale * 1024
        a["w"] += w * w_scale * 1024
        a["alg"] += sl["points"] * (sl["in_bytes"] + sl["out_bytes"])
    print("read bytes = %.4f x FETCH_SIZE x 1024, written bytes = %.4f x WRITE_SIZE x 1024 "
          "(the 1 GiB copy reads FETCH_SIZE %.0f KiB, writes WRITE_SIZE %.0f KiB)" % (f_scale, w_scale, cal_f or 0,
                                                                                    cal_w or 0))
    print("| Slot | Kernel | Read bytes | Written bytes | Algorithmic bytes | Measured / algorithmic |")
    print("|:--|:--|--:|--:|--:|--:|")
    for nm, a in agg.items():
        k = a["k"]
        print("| %s | %s | %.0f | %.0f | %.0f | %.2f |" % (nm, a["kernel"].replace("void fcc::", "").split("(")[0],
                                                           a["f"] / k, a["w"] / k, a["alg"] / k,
                                                           (a["f"] + a["w"]) / a["alg"]))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.summarize:
        summarize(args.summarize, args.workload + ("_fold" if args.fold else ""))
        return
    if args.workload in ("c1", "c2", "c4"):
        r = single_volume(args, args.workload)
    else:
        r = batched(args, args.workload)
    if r is None:  # --pmc-pass
        if args.copy_calibration:
            copy_calibration()
        return
    points, ms, dtype, cfg, roof, extra, cpu_case = r
    out = {
        "metric": "FCC-DCT points/s", "value": points / (ms * 1e-3), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg,
        "roofline": roof,
    }
    out.update(extra)
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cpu_case[0], cpu_case[1], args.cpu_seconds)
    print(json.dumps(out), flush=True)


def copy_calibration():
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
    b = a.clone()
    torch.cuda.synchronize()
    return int(b.numel() * 4)


if __name__ == "__main__":
    main()
