"""Benchmark of the EM plane sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--storage f32]

One step is one frame through the whole method, with inputs already resident
in HBM: lf_em_load (descriptors, ray prior, first weights, device-side input
validation), lf_em_iterate (all EM iterations of the configuration, one
fused launch) and lf_refocus (outputs stay in device memory).  The metric is
EM-iteration throughput H*W*D*K*I / t in G(pixel*disparity*view) per second
over the K timed steps, plus the p50/p99 of per-frame latency.

The roofline object refers to the dominant kernel (the fused EM iterations):
its algorithmic work is 6F + 12/K flops per (pixel, disparity, view) unit
and iteration (F = 2 descriptor components), its duration is measured with
HIP events on the stream it is launched on, and the peak is MI355X's FP32
vector rate.  The CPU baseline is the FP64 oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_HBM_GBS = 8000.0
F_DESC = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--storage", default=None, choices=["f32", "f16", "bf16"])
    ap.add_argument("--mode", default="soft", choices=["soft", "hard"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM traffic counters)")
    return ap.parse_args()


def log(args, msg):
    if not args.quiet:
        print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(spec, frame, storage, mode, budget_s):
    """The FP64 oracle as it stands, on the host cores, over whole frames of the
    same workload until about `budget_s` seconds of CPU work have elapsed."""
    import oracle as O
    p = O.make_params(spec.K, spec.H, spec.W, spec.ref, [float(np.float32(b)) for b in spec.baselines],
                      float(np.float32(spec.d_min)), float(np.float32(spec.d_step)), spec.D,
                      float(np.float32(frame.beta)), float("nan"), float(np.float32(spec.gamma)),
                      float(np.float32(spec.sigma)), float(np.float32(spec.tau)), storage, mode)
    O.lib()
    frames, t0 = 0, time.perf_counter()
    while True:
        r = O.reconstruct(p, frame.views, frame.S_P, frame.mu_T, spec.n_iters)
        frames += 1
        el = time.perf_counter() - t0
        if el >= budget_s or frames >= 50:
            break
    units = spec.H * spec.W * spec.D * spec.K * spec.n_iters * frames
    return {"value": units / el / 1e9, "unit": "EM-iter Gpix·disp·view/s", "cores": int(r["threads"]),
            "kind": "oracle", "sample": f"{frames} full frame(s) of the same workload, {el:.1f} s, FP64 C/OpenMP",
            "frames_per_s": frames / el}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "the per-GPU work shards by row bands, see the design notes.", file=sys.stderr)
        sys.exit(2)
    import torch
    import lf_scenes as S
    import paper_2003_11076_amd as LF

    spec = S.config_spec(args.config)
    storage = args.storage or spec.storage
    log(args, f"generating {spec.name} ({spec.W}x{spec.H}, K={spec.K}, D={spec.D}, I={spec.n_iters})")
    frame = S.make_frame(spec)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    views = torch.from_numpy(frame.views).to(dev)
    sp = torch.from_numpy(frame.S_P).to(dev)
    mu = torch.from_numpy(frame.mu_T).to(dev)
    K, H, W, D, I = spec.K, spec.H, spec.W, spec.D, spec.n_iters
    rgb = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    d_idx = torch.empty((H, W), dtype=torch.int32, device=dev)
    q = torch.empty((K, H, W), dtype=torch.float32, device=dev)
    hole = torch.empty((H, W), dtype=torch.uint8, device=dev)
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE
    p = LF.make_params(K, H, W, spec.ref, spec.baselines, spec.d_min, spec.d_step, D, frame.beta,
                       gamma=spec.gamma, sigma=spec.sigma, tau_init=spec.tau, storage=storage, mode=args.mode,
                       flags=flags)
    torch.cuda.synchronize()
    ctx = LF.lf_em_init(p, views, sp, mu, hip_stream=stream.cuda_stream)

    def step(ev=None):
        LF.lf_em_load(ctx, views, sp, mu)
        if ev is not None:
            ev[0].record(stream)
        LF.lf_em_iterate(ctx, I)
        if ev is not None:
            ev[1].record(stream)
        LF.lf_refocus(ctx, rgb, d_idx, q, hole, 0)

    if args.calib_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the
        # counters read for the EM kernel
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(args, f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(args, f"timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        step(evs[i])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    em_ms = np.array([a.elapsed_time(b) for a, b in evs])
    LF.lf_em_destroy(ctx)

    units = H * W * D * K * I
    value = units * args.steps / t_total / 1e9
    lat_ms = np.array(lat) * 1e3
    em_avg_s = float(em_ms.mean()) * 1e-3
    flops_per_unit = 6 * F_DESC + 12.0 / K
    achieved = flops_per_unit * units / em_avg_s / 1e12
    # algorithmic HBM bytes of the EM launch: descriptors, rho, q in and out,
    # mu_T, d_idx and the per-pixel objective, once per launch
    sf = 8 if storage == "f32" else 4
    em_bytes = H * W * (K * (sf + 4 + 4 + 4) + 4 + 4 + 4)
    out = {
        "metric": "EM-iter Gpix·disp·view/s",
        "value": value,
        "unit": "EM-iter Gpix·disp·view/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene generator, uint8 views, float32 S_P and mu_T)",
        "config": {"workload": spec.name, "K": K, "H": H, "W": W, "D": D, "em_iters": I, "storage": storage,
                   "mode": args.mode, "parallelism": "single-gpu"},
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "frames_per_s": args.steps / t_total,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None,
            "kernel": "lf_em_kernel",
            "kernel_ms": em_avg_s * 1e3,
            "flops_per_unit": flops_per_unit,
            "units_per_launch": units,
            "algorithmic_hbm_GBps": em_bytes / em_avg_s / 1e9,
        },
    }
    if not args.no_cpu_baseline:
        log(args, "timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(spec, frame, storage, args.mode, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
