#!/usr/bin/env python3
"""Throughput of the arbitrary-shape-surface Fresnel forward on one MI355X.

Workload: the 2048 x 2048 spherical-cap surface (R = 50 mm, 8 um pitch with
+-0.3 pitch jitter, binary amplitude mask with uniform phase, lambda = 532 nm,
z0 = 0.2 m, 2048 x 2048 destination at 8 um, sigma = 2, w = 7, tol 1e-5).
One step is the whole hot path over one batch of synthetic input already
resident in HBM: the FP64 pre-phase and tile binning (asf_setpts) and the
spreading plus both FFT passes with the fused deconvolution (asf_forward).
The line also reports the geometry-cached forward alone (``fwd``), the
adjoint of the same plan (``adjoint``, the type-2 direction used for gradients),
the one-dimensional path on a batch of the quadratic profile (``line_1d``) and one
training sample and one inference of the learned warm start (``warm_start``).

Prints one JSON line.  ``value`` is NU points/s (source points per second of
whole-step time) with FP32 FFT stages, the precision the 1e-5 bar is stated for;
the split-FP16 FFT is timed too and reported under ``variants``.  ``roofline``
covers the dominant kernel (the spread), timed with HIP events on the stream it
runs on, against 28 B per point plus 8 B per fine-grid cell; ``cpu_baseline``
times the CPU oracle (the direct sum, and its matrix-product form ``crop_gemm``)
on bounded samples on the host cores this job may use, and the GPU output is
compared with the oracle there and, where stored, on the full-size evaluation
sets (256^2 centre and corner crops, 4096 random pixels).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "spread_cap_2048_traffic.txt")
PROFILE_FFT = os.path.join(ROOT, "profiles", "fft_counters_cap_2048.txt")
CSRC = os.path.join(ROOT, "paper_1203_3583_amd", "csrc")
SPREAD_SOURCE = os.path.join(CSRC, "spread.hip")
FFT_SOURCE = os.path.join(CSRC, "fft.hip")
GOLDEN = os.path.join(ROOT, "tests", "golden", "make_eval_sets.py")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cap_2048", choices=sorted(WORKLOADS),
                    help="surface to time (the headline is cap_2048; the others are the small "
                         "and the large configuration)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-pixels", type=int, default=2048, help="oracle sample size (pixels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for counter calibration)")
    return ap.parse_args()


def algorithmic_spread_bytes(n_points, cells_written):
    """Per launch: 28 B per source point (u1 8 B and a 20 B record: point index 4,
    fine cell and offsets 8, pre-phase 8) plus 8 B per fine-grid cell written."""
    return 28 * n_points + 8 * cells_written


def cells_written(torch, plan):
    """Fine-grid cells the spreading writes: all of them, or, while the plan leaves the
    tiles no record reaches unwritten, the cells of the tiles the binning flags."""
    info = plan.info()
    if not info["skip_empty"]:
        return info["nfx"] * info["nfy"]
    flags = plan.workspace_view(info["off_live"], info["ntiles"], torch.uint8)
    return int(flags.sum().item()) * info["tile_x"] * info["tile_y"]


def _summary_fields(path):
    fields = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    return fields


def _code_sha(path):
    """SHA-256 of a C++/HIP source's code: comments removed and whitespace collapsed,
    so that a stored counter summary stays tied to the code it was measured on and
    not to the wording of its comments."""
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()


def stored_traffic():
    """HBM bytes per spread launch from the committed counter summary, if it was
    taken on the current spread code (else None)."""
    fields = _summary_fields(PROFILE_TRAFFIC)
    if fields.get("spread_code_sha256") != _code_sha(SPREAD_SOURCE):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stored_fft_busy():
    """Busy fraction of the unit each FFT pass computes on, from the committed counter
    summary (FP32 passes: vector ALU, SQ_ACTIVE_INST_VALU; split-FP16 passes: matrix
    cores, SQ_VALU_MFMA_BUSY_CYCLES; each over GRBM_GUI_ACTIVE and the SIMD count),
    if it was taken on the current FFT code (else None)."""
    fields = _summary_fields(PROFILE_FFT)
    if fields.get("fft_code_sha256") != _code_sha(FFT_SOURCE):
        return None
    out = {}
    for k, v in fields.items():
        if k.startswith("busy_"):
            try:
                out[k[len("busy_"):]] = float(v)
            except ValueError:
                pass
    return out or None


def eval_set_errors(name, u2_by_fft):
    """rel-L2 of each FFT precision's u2 on the stored evaluation sets of workload
    `name` (None if none are stored for it or they were computed from other inputs)."""
    import importlib.util
    import synth

    spec = importlib.util.spec_from_file_location("make_eval_sets", GOLDEN)
    g = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(g)
    if name not in g.CONFIGS or not os.path.exists(g.path_for(name)):
        return None
    sets, digest = g.load(name)
    if digest != g.input_digest(synth.config(name)):
        return None
    return {fft: {s: float(np.linalg.norm(u2[iy, ix] - v) / np.linalg.norm(v)) for s, (ix, iy, v) in sets.items()}
            for fft, u2 in u2_by_fft.items()}


def time_calls(torch, plan, fn, steps, warmup):
    """Average seconds per call of fn() (plan geometry cached), and its stage times."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    plan.set_timing(True)
    acc = {}
    for _ in range(steps):
        fn()
        for k, v in plan.stage_times().items():
            acc[k] = acc.get(k, 0.0) + v / steps
    plan.set_timing(False)
    return sec, acc


def line_bench(torch, asf, synth, steps, warmup, batch=4096):
    """The one-dimensional path: `batch` fields through the quadratic profile
    (1024 points, 1024 pixels), one launch per call, timed with HIP events on the
    stream the kernel runs on (torch's current stream)."""
    w = synth.line_config("quadratic_1d")
    rng = np.random.default_rng(2)
    u = rng.standard_normal((batch, w.n)) + 1j * rng.standard_normal((batch, w.n))
    u = torch.from_numpy(u.astype(np.complex64)).cuda()
    plan = asf.LinePlan(torch.from_numpy(w.x).cuda(), torch.from_numpy(w.d).cuda(), w.lam, w.z0, w.p2,
                        w.m, tol=w.tol, incident=w.incident)
    out = torch.empty((batch, w.m), dtype=torch.complex64, device=u.device)
    for _ in range(warmup):
        plan.forward(u, out=out)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        plan.forward(u, out=out)
    stop.record()
    torch.cuda.synchronize()
    sec = start.elapsed_time(stop) * 1e-3 / steps
    plan.close()
    alg = batch * 8 * (w.n + w.m)          # u1 read and u2 written once per field
    return {"workload": "quadratic profile (Sec. 3): 1024 points at 10 um arc pitch, 1024 pixels, "
                        "lambda=633nm, z0=1m", "batch": batch, "ms_per_call": sec * 1e3,
            "value": batch * w.n / sec, "unit": "NU points/s",
            "algorithmic_bytes": alg, "hbm_frac": alg / sec / (HBM_PEAK_GBS * 1e9)}


def warm_bench(torch, steps=3):
    """The learned warm start at its working size: one training sample of the
    encoder-decoder on a 512^2 problem (network forward, the diffraction forward and
    adjoint for the intensity loss, network backward), timed with HIP events."""
    import numpy as np
    import paper_1203_3583_amd.warmstart as ws

    pr = ws.HoloProblems(side=512, seed=0)
    d, inten, _ = pr.make(np.random.default_rng(1))
    net = ws.WarmNet(base=32, seed=0)

    def sample():
        out, cache = net.forward(pr.net_input(d, inten))
        loss, dphi = ws.physics_loss_and_grad(pr, d, inten, out[0, :, :, 0].contiguous())
        dout = torch.zeros_like(out)
        dout[0, :, :, 0] = dphi
        net.backward(dout, cache)
        return out

    sample()
    start, mid, stop = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    fwd = 0.0
    start.record()
    for _ in range(steps):
        sample()
    stop.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(stop) / steps
    start.record()
    for _ in range(steps):
        net.infer(pr.net_input(d, inten))
    stop.record()
    torch.cuda.synchronize()
    fwd = start.elapsed_time(stop) / steps
    # forward FLOPs of the 15 convolutions (2 per multiply-add) at 512^2 and below
    flops = 0
    hw = {0: 1, 1: 1, 2: 4, 3: 4, 4: 16, 5: 16, 6: 64, 7: 64, 8: 16, 9: 16, 10: 4, 11: 4, 12: 1, 13: 1, 14: 1}
    for i, (ci, co, _) in enumerate(net.shapes):
        flops += 2 * 9 * ci * co * (512 * 512 // hw[i])
    return {"workload": "encoder-decoder (4 levels, base 32) on a 512x512 phase-hologram problem",
            "train_sample_ms": total, "inference_ms": fwd,
            "inference_tflops": flops / (fwd * 1e-3) / 1e12, "unit": "ms per sample"}


WORKLOADS = {
    "cap_2048": "spherical cap R=50mm, 2048x2048 source at 8um (+-0.3 pitch jitter), binary-mask u1, "
                "lambda=532nm, z0=0.2m, 2048x2048 output at 8um",
    "sinusoid_4096": "sinusoidal relief 30um x 0.5mm period, 4096x4096 source at 4um (+-0.3 pitch jitter), "
                     "uniform u1, lambda=633nm, z0=0.3m, 4096x4096 output at 4um",
    "sinusoid_128": "sinusoidal relief 50um x 1mm period, 128x128 source at 8um (+-2.4um jitter), "
                    "uniform u1, lambda=532nm, z0=0.1m, 128x128 output at 8um",
}


def cpu_model() -> str:
    """The host CPU's model name (Linux), for the CPU baseline's record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth(torch, dev, nbytes=256 << 20, reps=20):
    """Achievable HBM bandwidth: a plain device-to-device copy of nbytes, counted as
    read plus write bytes per second (GB/s), timed with HIP events."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.copy_(a)
    stop.record()
    torch.cuda.synchronize()
    sec = start.elapsed_time(stop) * 1e-3 / reps
    del a, b
    return 2.0 * nbytes / sec / 1e9


def time_steps(torch, plan, x, y, d, u, out, steps, warmup, stage_events):
    for _ in range(warmup):
        plan.setpts(x, y, d)
        plan.forward(u, out=out)
    torch.cuda.synchronize()
    plan.set_timing(stage_events)
    stage_sum = {}
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.setpts(x, y, d)
        plan.forward(u, out=out)
        if stage_events:
            for k, v in plan.stage_times().items():
                stage_sum[k] = stage_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.set_timing(False)
    return dt / steps, {k: v / steps for k, v in stage_sum.items()}


def median_step_ms(torch, plan, x, y, d, u, out, steps):
    """Median over `steps` single steps, each bracketed by HIP events on the
    current stream (the steps run back to back; one synchronisation at the end)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        plan.setpts(x, y, d)
        plan.forward(u, out=out)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the forward is "
              "linear in the points, so a multi-GPU run would shard points and sum-reduce u2 -- "
              "that path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1203_3583_amd as asf

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    w = synth.config(args.workload)
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    d = torch.from_numpy(w.d).to(dev)
    u = torch.from_numpy(w.u).to(dev)
    out = torch.empty((w.my, w.mx), dtype=torch.complex64, device=dev)

    results = {}
    for fft in ("fp32", "split_fp16"):
        plan = asf.Plan(x, y, d, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, tol=w.tol, fft=fft)
        info = plan.info()
        sec, _ = time_steps(torch, plan, x, y, d, u, out, args.steps, args.warmup, False)
        med = median_step_ms(torch, plan, x, y, d, u, out, args.steps)
        _, stages = time_steps(torch, plan, x, y, d, u, out, args.steps, 0, True)
        cells = cells_written(torch, plan)
        plan.forward(u, out=out)
        torch.cuda.synchronize()
        u2 = out.cpu().numpy().astype(np.complex128)
        # the geometry-cached forward, and the adjoint (type-2 direction) of the same plan
        fwd_sec, fwd_stages = time_calls(torch, plan, lambda: plan.forward(u, out=out), args.steps, 2)
        g1 = torch.empty(w.n, dtype=torch.complex64, device=dev)
        adj_sec, adj_stages = time_calls(torch, plan, lambda: plan.adjoint(out, out=g1), args.steps, 2)
        results[fft] = {"sec": sec, "median_ms": med, "stages": stages, "info": info, "u2": u2, "cells": cells,
                        "fwd_sec": fwd_sec, "fwd_stages": fwd_stages,
                        "adj_sec": adj_sec, "adj_stages": adj_stages}
        plan.close()

    line = line_bench(torch, asf, synth, args.steps, args.warmup)
    warm = warm_bench(torch)
    copy_gbs = copy_bandwidth(torch, dev)

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    # FP32 FFT stages: the precision the 1e-5 bar of the metric is stated for
    head = "fp32"
    r = results[head]
    n = w.n
    info = r["info"]
    spread_ms = r["stages"].get("spread")
    alg = algorithmic_spread_bytes(n, r["cells"])
    achieved = alg / (spread_ms * 1e-3) / 1e9 if spread_ms else None
    line = {
        "metric": "NU points/s, 2D forward at rel-L2<=1e-5 vs FP64 oracle",
        "value": n / r["sec"],
        "unit": "NU points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["sec"] * 1e3,
        # the same step timed one at a time with HIP events: the median of `steps`
        "median_ms_per_step": r["median_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "n_points": n, "fine_grid": [info["nfy"], info["nfx"]], "w": info["w"],
                   "sigma": 2, "fft": head, "step": "setpts(prephase+bin) + forward(spread+fft+deconv)"},
        "stages_ms": {k: round(v, 4) for k, v in r["stages"].items()},
        # split_fp16: FFT stages as FP16 hi+lo products on the matrix cores (bar 1e-4)
        "variants": {k: {"ms_per_step": v["sec"] * 1e3, "median_ms_per_step": v["median_ms"], "value": n / v["sec"],
                         "stages_ms": {s: round(t, 4) for s, t in v["stages"].items()},
                         "fwd_ms": v["fwd_sec"] * 1e3, "adjoint_ms": v["adj_sec"] * 1e3}
                     for k, v in results.items()},
        # geometry cached (plan reused): the forward alone, and the adjoint g1 = A^H g2
        "fwd": {"ms_per_call": r["fwd_sec"] * 1e3, "value": n / r["fwd_sec"], "unit": "NU points/s",
                "stages_ms": {s: round(t, 4) for s, t in r["fwd_stages"].items()}},
        "adjoint": {"ms_per_call": r["adj_sec"] * 1e3, "value": n / r["adj_sec"], "unit": "NU points/s",
                    "stages_ms": {s: round(t, 4) for s, t in r["adj_stages"].items()}},
        "line_1d": line,
        "warm_start": warm,
        "roofline": {
            "kernel": "spread",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            # a plain 256 MiB device copy on the same GPU: the bandwidth reachable in practice
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs if achieved else None,
            # counter traffic was taken on the cap's spread only
            "traffic": stored_traffic() if args.workload == "cap_2048" else None,
            "algorithmic_bytes": alg,
            "bytes_model": "28 B per point (u1 8 + record 20) + 8 B per fine cell written",
            "fine_cells_written": r["cells"],
            "avg_launch_ms": spread_ms,
        },
        # busy fraction of the FFT passes' compute unit (vector ALU for FP32, matrix
        # cores for split FP16), from the committed counter summary
        "fft_unit_busy": stored_fft_busy() if args.workload == "cap_2048" else None,
        # rel-L2 against the FP64 oracle on the stored evaluation sets (both precisions)
        "rel_l2_eval_sets": eval_set_errors(args.workload, {k: v["u2"] for k, v in results.items()}),
        "cpu_baseline": None,
    }

    if not args.no_cpu:
        import oracle  # CPU baseline leg only

        # every core this job may run on (the OpenMP default, which OMP_NUM_THREADS caps)
        threads = oracle.threads(0)
        ix, iy = synth.sample_pixels(w.mx, w.my, args.cpu_pixels, seed=11)
        t0 = time.perf_counter()
        ref = oracle.direct(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, ix, iy,
                            incident=w.incident, nthreads=threads)
        t_cpu = time.perf_counter() - t0
        t_full = t_cpu * (w.mx * w.my) / len(ix)
        # the matrix-product form of the same sum on a 64 x 64 centre crop
        crop = 64
        cx, cy = w.mx // 2 - crop // 2, w.my // 2 - crop // 2
        t0 = time.perf_counter()
        oracle.crop_gemm(w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my,
                         range(cx, cx + crop), range(cy, cy + crop), incident=w.incident, nthreads=threads)
        t_gemm = time.perf_counter() - t0
        try:
            affinity = len(os.sched_getaffinity(0))
        except AttributeError:
            affinity = os.cpu_count()
        line["cpu_baseline"] = {
            "value": n / t_full,
            "unit": "NU points/s",
            "cores": threads,
            "nproc": os.cpu_count(),
            "affinity_cores": affinity,
            "cpu": cpu_model(),
            "kind": "oracle",
            "sample": f"{len(ix)} random destination pixels of the {w.mx}x{w.my} grid, each a direct FP64 "
                      f"sum over all {n} points ({t_cpu:.1f} s on {threads} threads), extrapolated to the full grid",
            "terms_per_s": n * len(ix) / t_cpu,
            "crop_gemm": {"value": n / (t_gemm * (w.mx * w.my) / (crop * crop)), "unit": "NU points/s",
                          "terms_per_s": n * crop * crop / t_gemm,
                          "sample": f"{crop}x{crop} centre crop over all {n} points ({t_gemm:.1f} s), "
                                    "extrapolated to the full grid"},
        }
        line["rel_l2_vs_oracle_sample"] = {
            k: float(np.linalg.norm(v["u2"][iy, ix] - ref) / np.linalg.norm(ref)) for k, v in results.items()}

    print(json.dumps(line))


if __name__ == "__main__":
    main()
