"""Benchmark of the EM plane sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain] [--storage f32]

One step is one frame through the whole method, with inputs already resident
in HBM: lf_em_load (descriptors, ray prior, first weights, device-side input
validation), lf_em_iterate (all EM iterations of the configuration, one
fused launch) and lf_refocus (outputs stay in device memory).  The metric is
EM-iteration throughput H*W*D*K*I / t in G(pixel*disparity*view) per second
over the K timed steps, plus the p50/p99 of per-frame latency.

The timed frames are dealt round robin to --streams contexts (default 2),
each on its own HIP stream, so that one frame's kernels start while the last
waves of the previous frame's EM launch are still finishing.  Latency is
taken separately, one frame at a time on an otherwise idle GPU.

The roofline object refers to the dominant kernel (the fused EM iterations):
its algorithmic work is 6F + 12/K flops per (pixel, disparity, view) unit
and iteration (F = 2 descriptor components), its duration is measured with
HIP events on the stream it is launched on, in the one-frame-at-a-time loop
(a launch alone on the GPU), and the peak is MI355X's FP32 vector rate.  The
CPU baseline is the FP64 oracle on the host cores.
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
ROOT = os.path.dirname(os.path.abspath(__file__))
# sources of the EM kernel: HBM traffic measured with rocprofv3 counters is
# reported only while these are unchanged since the measurement
def _em_sources():
    import glob
    csrc = os.path.join(ROOT, "paper_2003_11076_amd", "csrc")
    names = sorted(glob.glob(os.path.join(csrc, "lf_em*.hip")) + glob.glob(os.path.join(csrc, "lf_em*.h")))
    return [os.path.relpath(n, ROOT) for n in names]


def measured_traffic(workload):
    """HBM bytes per EM launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload (scaled by a plain copy's counters),
    or None when there is none or the kernel changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"lf_em_kernel_{workload}.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in _em_sources():
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest()[:16] != rec.get("src_hash"):
        return None
    return rec.get("traffic_bytes")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="plain", choices=["small", "plain", "precision", "large"])
    ap.add_argument("--streams", type=int, default=2,
                    help="contexts (one HIP stream each) the timed frames are dealt to, round robin")
    ap.add_argument("--storage", default=None, choices=["f32", "f16", "bf16"])
    ap.add_argument("--mode", default="soft", choices=["soft", "hard"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the frame-server legs")
    ap.add_argument("--no-variants", action="store_true", help="skip the variant legs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM traffic counters)")
    return ap.parse_args()


def log(args, msg):
    if not args.quiet:
        print(f"[bench] {msg}", file=sys.stderr, flush=True)


def variant_legs(LF, torch, spec, frame, storage, views, sp, mu, stream, reps=20):
    """EM launch time of the same frame with the paper's speed levers and
    E-step forms: the search window around mu_T, dynamic reference pixels
    only, both, and the enumeration E-step."""
    K, H, W, D, I = spec.K, spec.H, spec.W, spec.D, spec.n_iters
    legs = [("window_3sigma", "soft", LF.LF_PRIOR_WINDOW), ("dynamic_only", "soft", LF.LF_DYNAMIC_ONLY),
            ("window_and_dynamic_only", "soft", LF.LF_PRIOR_WINDOW | LF.LF_DYNAMIC_ONLY),
            ("enumeration_soft", "enum_soft", 0), ("enumeration_hard", "enum_hard", 0)]
    out = {}
    dev_flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE
    for name, mode, flags in legs:
        p = LF.make_params(K, H, W, spec.ref, spec.baselines, spec.d_min, spec.d_step, D, frame.beta,
                           gamma=spec.gamma, sigma=spec.sigma, tau_init=spec.tau, storage=storage, mode=mode,
                           flags=dev_flags | flags)
        ctx = LF.lf_em_init(p, views, sp, mu, hip_stream=stream.cuda_stream)
        ts = []
        for r in range(reps + 3):
            LF.lf_em_load(ctx, views, sp, mu)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            LF.lf_em_iterate(ctx, I)
            e1.record(stream)
            torch.cuda.synchronize()
            if r >= 3:
                ts.append(e0.elapsed_time(e1))
        LF.lf_em_destroy(ctx)
        out[name] = {"em_ms": float(np.median(ts)), "mode": mode}
    return out


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


# ---------------------------------------------------------------------------
# Serving leg: the frame server under the 16-stream mix, and on the bench
# workload's frames for a like-for-like comparison with the plain path.
# ---------------------------------------------------------------------------

def _frame_arrays(spec):
    import lf_scenes as S
    fr = S.make_frame(spec)
    return spec, fr.views, fr.S_P, fr.mu_T, fr.beta


def _make_frames(specs, workers):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_frame_arrays, specs))


class _Driver:
    """Submits frames to a server from a few threads (submission copies the
    inputs) and keeps each frame's output arrays alive until it completes."""

    def __init__(self, LF, srv, frames, storage):
        import queue
        import threading
        self.LF, self.srv, self.frames = LF, srv, frames
        self.params = []
        for spec, views, sp, mu, beta in frames:
            self.params.append(LF.make_params(spec.K, spec.H, spec.W, spec.ref, spec.baselines, spec.d_min,
                                              spec.d_step, spec.D, beta, gamma=spec.gamma, sigma=spec.sigma,
                                              tau_init=spec.tau, storage=storage))
        self.lock = threading.Lock()
        self.live = {}
        self.done_q = queue.Queue()
        self._cb = LF.lf_done_fn(self._on_done)

    def _on_done(self, fid, status, user):
        self.done_q.put((fid, status))

    def submit(self, stream, idx):
        import time as _t
        spec, views, sp, mu, _ = self.frames[idx]
        out = (np.empty((spec.H, spec.W, 3), np.float32), np.empty((spec.H, spec.W), np.int32))
        while True:
            try:
                fid = self.LF.lf_submit_frame(self.srv, stream, self.params[idx], views, sp, mu, out[0], out[1],
                                              None, self._cb)
                break
            except self.LF.LFError as e:
                if e.status != self.LF.LF_EAGAIN:
                    raise
                _t.sleep(0.0002)
        with self.lock:
            self.live[fid] = (stream, out)
        return fid

    def wait_one(self):
        fid, status = self.done_q.get()
        assert status == 0, status
        with self.lock:
            stream, _ = self.live.pop(fid)
        return fid, stream


def _units(spec, n_iters):
    return spec.H * spec.W * spec.D * spec.K * n_iters


SERVE_STREAMS = 16


def serving_frames(S, log_fn):
    """Two frames of each of the 16 mix streams.  Generated in worker
    processes before this process touches the GPU (the workers are forked)."""
    log_fn(f"serving: generating 2 frames for each of {SERVE_STREAMS} streams")
    specs = [S.serving_stream_spec(s, f) for s in range(SERVE_STREAMS) for f in range(2)]
    return _make_frames(specs, min(8, os.cpu_count() or 1))


def serve_leg(args, LF, frames, log_fn):
    import random
    from concurrent.futures import ThreadPoolExecutor
    n_streams = SERVE_STREAMS
    n_iters = frames[0][0].n_iters
    budget = 1 << 30
    srv = LF.lf_server_create(budget, n_streams, n_iters, 3 << 30)
    drv = _Driver(LF, srv, frames, "f16")
    idx_of = lambda stream, k: 2 * stream + (k % 2)
    pool = ThreadPoolExecutor(max_workers=4)
    try:
        # warm-up: one frame per stream
        for st in range(n_streams):
            drv.submit(st, idx_of(st, 0))
        LF.lf_server_drain(srv)
        while not drv.done_q.empty():
            drv.wait_one()
        # saturation: closed loop, two frames outstanding per stream
        per_stream = 12
        LF.lf_server_reset_stats(srv)
        sent = {st: 0 for st in range(n_streams)}
        futs = []
        t0 = time.perf_counter()
        for st in range(n_streams):
            for _ in range(2):
                futs.append(pool.submit(drv.submit, st, idx_of(st, sent[st])))
                sent[st] += 1
        completed, units = 0, 0
        total = n_streams * per_stream
        while completed < total:
            fid, st = drv.wait_one()
            completed += 1
            units += _units(frames[idx_of(st, 0)][0], n_iters)
            if sent[st] < per_stream:
                futs.append(pool.submit(drv.submit, st, idx_of(st, sent[st])))
                sent[st] += 1
        t_sat = time.perf_counter() - t0
        for f in futs:
            f.result()
        sat = LF.lf_server_stats(srv)
        fps_sat = total / t_sat
        log_fn(f"serving: saturation {fps_sat:.0f} frames/s, p99 {sat.p99_ms:.2f} ms")
        # open loop: Poisson arrivals at 0.7 x saturation over the 16 streams
        rate = 0.7 * fps_sat
        n_frames = max(200, int(rate * 3.0))
        rng = random.Random(7)
        LF.lf_server_reset_stats(srv)
        futs, t = [], 0.0
        t0 = time.perf_counter()
        counter = {st: 0 for st in range(n_streams)}
        for i in range(n_frames):
            t += rng.expovariate(rate)
            st = rng.randrange(n_streams)
            k = counter[st]
            counter[st] += 1
            delay = t0 + t - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            futs.append(pool.submit(drv.submit, st, idx_of(st, k)))
        for f in futs:
            f.result()
        LF.lf_server_drain(srv)
        t_open = time.perf_counter() - t0
        units_open = 0
        while not drv.done_q.empty():
            _, st = drv.wait_one()
            units_open += _units(frames[idx_of(st, 0)][0], n_iters)
        op = LF.lf_server_stats(srv)
    finally:
        pool.shutdown(wait=True)
        LF.lf_server_destroy(srv)
    return {
        "workload": "serving-mix-fp16-i8: 16 streams, 320x240/640x480/1280x960 (5/8/3 streams), K 3/5/7, "
                    "D 32/64/128, objects moving 2 px/frame, warm start per stream",
        "hbm_budget_bytes": budget,
        "saturation": {"frames_per_s": fps_sat, "gunits_per_s": units / t_sat / 1e9, "p50_ms": sat.p50_ms,
                       "p99_ms": sat.p99_ms, "mean_batch_frames": sat.mean_batch_frames, "frames": total},
        "poisson_0.7": {"offered_frames_per_s": rate, "frames_per_s": op.completed / t_open,
                        "gunits_per_s": units_open / t_open / 1e9, "p50_ms": op.p50_ms, "p99_ms": op.p99_ms,
                        "mean_batch_frames": op.mean_batch_frames, "frames": int(op.completed),
                        "hbm_peak_bytes": int(op.hbm_peak)},
    }


def serve_same_workload(args, LF, frame, spec, n_frames=200, n_streams=4):
    """The bench workload's frame through the FP16 frame server (streams in a
    closed loop): frames/s and latency beside the plain path's."""
    from concurrent.futures import ThreadPoolExecutor
    frames = [(spec, frame.views, frame.S_P, frame.mu_T, frame.beta)]
    srv = LF.lf_server_create(2 << 30, n_streams, spec.n_iters, 1 << 30)
    drv = _Driver(LF, srv, frames, "f16")
    pool = ThreadPoolExecutor(max_workers=4)
    try:
        for st in range(n_streams):
            drv.submit(st, 0)
        LF.lf_server_drain(srv)
        while not drv.done_q.empty():
            drv.wait_one()
        LF.lf_server_reset_stats(srv)
        sent = {st: 0 for st in range(n_streams)}
        per = n_frames // n_streams
        futs = []
        t0 = time.perf_counter()
        for st in range(n_streams):
            for _ in range(2):
                futs.append(pool.submit(drv.submit, st, 0))
                sent[st] += 1
        done = 0
        while done < per * n_streams:
            _, st = drv.wait_one()
            done += 1
            if sent[st] < per:
                futs.append(pool.submit(drv.submit, st, 0))
                sent[st] += 1
        dt = time.perf_counter() - t0
        for f in futs:
            f.result()
        stt = LF.lf_server_stats(srv)
    finally:
        pool.shutdown(wait=True)
        LF.lf_server_destroy(srv)
    units = spec.H * spec.W * spec.D * spec.K * spec.n_iters
    return {"storage": "f16", "streams": n_streams, "frames_per_s": done / dt,
            "gunits_per_s": units * done / dt / 1e9, "p50_ms": stt.p50_ms, "p99_ms": stt.p99_ms,
            "mean_batch_frames": stt.mean_batch_frames,
            "note": "host inputs and outputs (PCIe copies included), unlike the plain-path line"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "the per-GPU work shards by row bands, see the design notes.", file=sys.stderr)
        sys.exit(2)
    import torch
    import lf_scenes as S
    import paper_2003_11076_amd as LF

    spec = S.workload_spec(args.workload)
    storage = args.storage or spec.storage
    log(args, f"generating {spec.name} ({spec.W}x{spec.H}, K={spec.K}, D={spec.D}, I={spec.n_iters})")
    frame = S.make_frame(spec)
    serve = not args.no_serving and args.workload == "plain"
    mix_frames = serving_frames(S, lambda m: log(args, m)) if serve else None
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    views = torch.from_numpy(frame.views).to(dev)
    sp = torch.from_numpy(frame.S_P).to(dev)
    mu = torch.from_numpy(frame.mu_T).to(dev)
    K, H, W, D, I = spec.K, spec.H, spec.W, spec.D, spec.n_iters
    # device-resident inputs and outputs; the value check of the inputs is
    # read once after the timed frames instead of after each load, so frames
    # queue back to back on the streams
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE | LF.LF_DEFERRED_CHECK
    p = LF.make_params(K, H, W, spec.ref, spec.baselines, spec.d_min, spec.d_step, D, frame.beta,
                       gamma=spec.gamma, sigma=spec.sigma, tau_init=spec.tau, storage=storage, mode=args.mode,
                       flags=flags)
    n_streams = max(1, args.streams)
    # default-priority streams; stream 0 is the current one
    streams = [stream] + [torch.cuda.Stream(device=dev) for _ in range(n_streams - 1)]
    torch.cuda.synchronize()
    ctxs, outs = [], []
    for st in streams:
        ctxs.append(LF.lf_em_init(p, views, sp, mu, hip_stream=st.cuda_stream))
        outs.append((torch.empty((H, W, 3), dtype=torch.float32, device=dev),
                     torch.empty((H, W), dtype=torch.int32, device=dev),
                     torch.empty((K, H, W), dtype=torch.float32, device=dev),
                     torch.empty((H, W), dtype=torch.uint8, device=dev)))

    def step(i, ev=None):
        ctx, out, st = ctxs[i % n_streams], outs[i % n_streams], streams[i % n_streams]
        LF.lf_em_load(ctx, views, sp, mu)
        if ev is not None:
            ev[0].record(st)
        LF.lf_em_iterate(ctx, I)
        if ev is not None:
            ev[1].record(st)
        LF.lf_refocus(ctx, *out, 0)

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
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    log(args, f"timing {args.steps} steps over {n_streams} stream(s)")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    for ctx in ctxs:
        LF.lf_em_check(ctx)                   # the inputs of every timed frame were valid
    # one frame at a time on an otherwise idle GPU: latency, and the EM
    # launch's duration (HIP events on its stream) for the roofline
    n_lat = min(args.steps, 100)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
    lat = []
    for i in range(n_lat):
        t0 = time.perf_counter()
        step(0, evs[i])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    em_ms = np.array([a.elapsed_time(b) for a, b in evs])
    for ctx in ctxs:
        LF.lf_em_check(ctx)
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
                   "mode": args.mode, "parallelism": "single-gpu", "streams": n_streams},
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "frames_per_s": args.steps / t_total,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(spec.name) if storage == spec.storage and args.mode == "soft" else None,
            "kernel": "lf_em_kernel",
            "kernel_ms": em_avg_s * 1e3,
            "flops_per_unit": flops_per_unit,
            "units_per_launch": units,
            "algorithmic_hbm_GBps": em_bytes / em_avg_s / 1e9,
        },
    }
    if not args.no_variants:
        log(args, "timing the variants (search window, dynamic-only, enumeration)")
        out["variants"] = variant_legs(LF, torch, spec, frame, storage, views, sp, mu, stream)
        out["variants"]["plain_em_ms"] = em_avg_s * 1e3
    if serve:
        log(args, "serving the same workload through the FP16 frame server")
        out["serving_same_workload"] = serve_same_workload(args, LF, frame, spec)
        out["serving"] = serve_leg(args, LF, mix_frames, lambda m: log(args, m))
    if not args.no_cpu_baseline:
        log(args, "timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(spec, frame, storage, args.mode, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
