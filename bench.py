"""Benchmark of the EM plane sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain] [--storage f32]

One step is one frame through the whole method, with inputs already resident
in HBM: lf_em_load (descriptors, ray prior, first weights, device-side input
validation), lf_em_iterate (all EM iterations of the configuration, one
fused launch) and lf_refocus (outputs stay in device memory).  The metric is
EM-iteration throughput H*W*D*K*I / t in G(pixel*disparity*view) per second
over the K timed steps, plus the p50/p99 of per-frame latency over at least
100 frames taken one at a time on an otherwise idle GPU.

The timed frames are dealt round robin to --streams contexts, each on its
own HIP stream.  The JSON line carries, beside the headline workload (FP32
storage):
  forms         the precision workload (FP16 storage) and the large workload
                (BF16 storage), each with its own value, latency and roofline;
  serving_*     the FP16 frame server on the headline frame and on the
                16-stream serving mix (device-resident inputs and outputs;
                saturation and Poisson arrivals at 0.3/0.5/0.7/0.9 of it),
                and the mix with host buffers (PCIe copies included);
  large_concurrent  four large-workload streams in one server launch (BF16)
                beside the plain FP32 context on the same frames;
  variants      the work-avoiding variants and the enumeration E-step;
  cpu_baseline  the FP64 oracle on the host cores.

The roofline object refers to the dominant kernel (the fused EM
iterations): its algorithmic work is 6F + 12/K flops per (pixel, disparity,
view) unit and iteration (F = 2 descriptor components), the work of the full
sweep over every level; its duration is measured with HIP events on the
stream it is launched on; the peak is MI355X's FP32 vector rate.  The
`executed` part counts only what the hardware issued: the share of the full
sweep's level evaluations the prior-bounded sweep took (a diagnostic launch
with a counter), and the VALU issue share from the committed rocprofv3 SQ
counters while the kernel sources are unchanged.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector, packed (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_FP32_UNPACKED = 78.65    # without packed FP32 instructions, which every build here disables
PEAK_HBM_GBS = 8000.0
SIMDS, CLOCK_HZ = 1024, 2.4e9
F_DESC = 2
SERVE_STREAMS = 16


# ---------------------------------------------------------------------------
# Committed profile figures, used only while the kernel sources are unchanged
# ---------------------------------------------------------------------------

def _em_sources():
    import glob
    csrc = os.path.join(ROOT, "paper_2003_11076_amd", "csrc")
    names = sorted(glob.glob(os.path.join(csrc, "lf_em*.hip")) + glob.glob(os.path.join(csrc, "lf_em*.h")))
    return [os.path.relpath(n, ROOT) for n in names]


def em_src_hash():
    h = hashlib.sha256()
    for src in _em_sources():
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_record(workload, what):
    """profiles/lf_em_kernel_<workload>.<what>.json when its source hash is
    the current one, else None."""
    path = os.path.join(ROOT, "profiles", f"lf_em_kernel_{workload}.{what}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    return rec if rec.get("src_hash") == em_src_hash() else None


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
    ap.add_argument("--latency-frames", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision and large workloads")
    ap.add_argument("--no-serving", action="store_true", help="skip the frame-server legs")
    ap.add_argument("--no-variants", action="store_true", help="skip the variant legs")
    ap.add_argument("--poisson-frames", type=int, default=10000, help="frames per Poisson load level")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM traffic counters)")
    return ap.parse_args()


def log(args, msg):
    if not args.quiet:
        print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(v, q):
    return float(np.percentile(np.asarray(v, np.float64), q)) if len(v) else None


# ---------------------------------------------------------------------------
# Inputs: generated in worker processes before this process touches the GPU
# ---------------------------------------------------------------------------

def _frame_arrays(spec):
    import lf_scenes as S
    fr = S.make_frame(spec)
    return spec, fr.views, fr.S_P, fr.mu_T, float(fr.beta)


def make_inputs(args):
    import lf_scenes as S
    from concurrent.futures import ProcessPoolExecutor
    specs = {"main": [S.workload_spec(args.workload)]}
    if not args.no_forms:
        specs["precision"] = [S.workload_spec("precision")]
        # four streams of the large workload: the dynamic objects 2 px further in each
        specs["large"] = [S.workload_spec("large", dyn_shift=2.0 * i) for i in range(4)]
    if not args.no_serving:
        specs["mix"] = [S.serving_stream_spec(s, f) for s in range(SERVE_STREAMS) for f in range(2)]
    flat = [(k, i, sp) for k, v in specs.items() for i, sp in enumerate(v)]
    log(args, f"generating {len(flat)} frames ({', '.join(f'{k}: {len(v)}' for k, v in specs.items())})")
    with ProcessPoolExecutor(max_workers=min(8, len(flat))) as ex:
        arrs = list(ex.map(_frame_arrays, [sp for _, _, sp in flat]))
    out = {k: [None] * len(v) for k, v in specs.items()}
    for (k, i, _), a in zip(flat, arrs):
        out[k][i] = a
    return out


# ---------------------------------------------------------------------------
# Plain context legs
# ---------------------------------------------------------------------------

def _params(LF, spec, beta, storage, mode="soft", flags=0):
    return LF.make_params(spec.K, spec.H, spec.W, spec.ref, spec.baselines, spec.d_min, spec.d_step, spec.D, beta,
                          gamma=spec.gamma, sigma=spec.sigma, tau_init=spec.tau, storage=storage, mode=mode,
                          flags=flags)


def _to_dev(torch, arrs, dev):
    spec, views, sp, mu, beta = arrs
    return (torch.from_numpy(views).to(dev), torch.from_numpy(sp).to(dev), torch.from_numpy(mu).to(dev))


def form_leg(args, LF, torch, arrs, storage, steps, warmup, n_streams, mode="soft"):
    """Throughput of whole frames on n_streams contexts, latency of single
    frames, the EM launch's duration and the roofline of the EM kernel."""
    spec, _, _, _, beta = arrs
    dev = torch.device("cuda:0")
    views, sp, mu = _to_dev(torch, arrs, dev)
    K, H, W, D, I = spec.K, spec.H, spec.W, spec.D, spec.n_iters
    # device-resident inputs and outputs; the value check of the inputs is
    # read once after the timed frames instead of after each load, so frames
    # queue back to back on the streams
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE | LF.LF_DEFERRED_CHECK
    p = _params(LF, spec, beta, storage, mode, flags)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream(device=dev) for _ in range(n_streams - 1)]
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

    try:
        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        evs_t = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        ref = torch.cuda.Event(enable_timing=True)
        t_start = time.perf_counter()
        ref.record(streams[0])
        for i in range(steps):
            step(i, evs_t[i])
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t_start
        for ctx in ctxs:
            LF.lf_em_check(ctx)                   # the inputs of every timed frame were valid
        em_timed = np.array([a.elapsed_time(b) for a, b in evs_t])
        # time the GPU runs an EM launch (on either stream) per step: the
        # union of the launches' intervals, which overlap on two streams
        iv = sorted((ref.elapsed_time(a), ref.elapsed_time(b)) for a, b in evs_t)
        busy, cur = 0.0, None
        for s0, s1 in iv:
            if cur is None or s0 > cur[1]:
                if cur is not None:
                    busy += cur[1] - cur[0]
                cur = [s0, s1]
            else:
                cur[1] = max(cur[1], s1)
        busy += cur[1] - cur[0]
        em_busy_per_step = busy / steps
        # one frame at a time on an otherwise idle GPU: latency, and the EM
        # launch's duration alone
        n_lat = max(args.latency_frames, 1)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
        lat = []
        for i in range(n_lat):
            t0 = time.perf_counter()
            step(0, evs[i])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        em_alone = np.array([a.elapsed_time(b) for a, b in evs])
        # levels the sweeps took (an untimed diagnostic launch of the same frame)
        LF.lf_em_load(ctxs[0], views, sp, mu)
        level_steps = LF.lf_em_sweep_count(ctxs[0], I)
        for ctx in ctxs:
            LF.lf_em_check(ctx)
    finally:
        for ctx in ctxs:
            LF.lf_em_destroy(ctx)

    units = H * W * D * K * I
    lat_ms = np.array(lat) * 1e3
    # the EM launch's average duration over the timed region
    em_s = float(em_timed.mean()) * 1e-3
    em_alone_s = float(em_alone.mean()) * 1e-3
    flops_per_unit = 6 * F_DESC + 12.0 / K
    achieved = flops_per_unit * units / em_s / 1e12
    swept = 64.0 * level_steps / (H * W * D * I)
    sf = 8 if storage == "f32" else 4
    # algorithmic HBM bytes of the EM launch: descriptors, rho, 1 - rho, q in
    # and out, mu_T, d_idx and the per-pixel objective, once per launch
    em_bytes = H * W * (K * (sf + 4 + 4 + 4 + 4) + 4 + 4 + 4)
    traffic = profile_record(spec.name, "traffic") if storage == spec.storage and mode == "soft" else None
    sq = profile_record(spec.name, "sq") if storage == spec.storage and mode == "soft" else None
    executed = {
        "sweep_level_share": swept,
        "executed_TFLOPs": achieved * swept,
        "frac_executed_of_unpacked_peak": achieved * swept / PEAK_FP32_UNPACKED,
        "valu_issue_share": (sq["valu_insts"] * 4.0 / (SIMDS * CLOCK_HZ * sq["kernel_us"] * 1e-6)) if sq else None,
        "note": "sweep_level_share = 64 * level steps / (H*W*D*I) from lf_em_sweep_count; valu_issue_share = "
                "SQ_INSTS_VALU * 4 cycles / (1024 SIMDs * 2.4 GHz * kernel time) from the committed rocprofv3 "
                "counters of these kernel sources",
    }
    return {
        "workload": spec.name, "storage": storage, "mode": mode, "K": K, "H": H, "W": W, "D": D, "em_iters": I,
        "streams": n_streams, "steps": steps,
        "value": units * steps / t_total / 1e9,
        "ms_per_step": t_total / steps * 1e3,
        "frames_per_s": steps / t_total,
        "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99), "latency_frames": len(lat_ms),
        "em_ms_timed_region": float(em_timed.mean()),
        "em_busy_ms_per_step": em_busy_per_step,
        "em_ms_alone": em_alone_s * 1e3,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic["traffic_bytes"] if traffic else None,
            "kernel": "lf_em_kernel",
            "kernel_ms": em_s * 1e3,
            "kernel_ms_alone": em_alone_s * 1e3,
            "achieved_per_busy_time": flops_per_unit * units / (em_busy_per_step * 1e-3) / 1e12,
            "timing": "kernel_ms: average EM launch over the timed steps (HIP events on each launch's stream; "
                      "launches of the two streams overlap); kernel_ms_alone: one frame at a time on an idle GPU; "
                      "achieved_per_busy_time: the same work over the time an EM launch runs on either stream, "
                      "per step (em_busy_ms_per_step <= ms_per_step)",
            "flops_per_unit": flops_per_unit,
            "units_per_launch": units,
            "peak_unpacked": PEAK_FP32_UNPACKED,
            "frac_of_unpacked": achieved / PEAK_FP32_UNPACKED,
            "algorithmic_hbm_GBps": em_bytes / em_s / 1e9,
            "executed": executed,
        },
    }


def variant_legs(LF, torch, arrs, storage, reps=20, names=None):
    """EM launch time of the same frame, one launch at a time on an idle GPU,
    plain and with the paper's speed levers and E-step forms: the search
    window around mu_T, dynamic reference pixels only, both, and the
    enumeration E-step."""
    spec, _, sp_host, _, beta = arrs
    dev = torch.device("cuda:0")
    views, sp, mu = _to_dev(torch, arrs, dev)
    stream = torch.cuda.current_stream()
    legs = [("plain", "soft", 0), ("window_3sigma", "soft", LF.LF_PRIOR_WINDOW),
            ("dynamic_only", "soft", LF.LF_DYNAMIC_ONLY),
            ("window_and_dynamic_only", "soft", LF.LF_PRIOR_WINDOW | LF.LF_DYNAMIC_ONLY),
            ("enumeration_soft", "enum_soft", 0), ("enumeration_hard", "enum_hard", 0)]
    if names is not None:
        legs = [leg for leg in legs if leg[0] in names]
    out = {"workload": spec.name,
           # reference pixels whose static prior is below tau (the reference
           # view's ray lands on its own pixel, so rho_ref is S_P there)
           "dynamic_fraction": float(np.mean(sp_host[spec.ref] < np.float32(spec.tau)))}
    dev_flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE
    for name, mode, flags in legs:
        ctx = LF.lf_em_init(_params(LF, spec, beta, storage, mode, dev_flags | flags), views, sp, mu,
                            hip_stream=stream.cuda_stream)
        ts = []
        for r in range(reps + 3):
            LF.lf_em_load(ctx, views, sp, mu)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            LF.lf_em_iterate(ctx, spec.n_iters)
            e1.record(stream)
            torch.cuda.synchronize()
            if r >= 3:
                ts.append(e0.elapsed_time(e1))
        LF.lf_em_destroy(ctx)
        out[name] = {"em_ms": float(np.median(ts)), "mode": mode}
    if "plain" in out and "dynamic_only" in out:
        out["dynamic_only_time_share"] = out["dynamic_only"]["em_ms"] / out["plain"]["em_ms"]
    return out


# ---------------------------------------------------------------------------
# Frame server legs
# ---------------------------------------------------------------------------

class Frames:
    """Device-resident (or host) inputs of a set of frames and a ring of
    output buffers per stream for frames in flight."""

    def __init__(self, LF, torch, frames, storage, device_io, ring=16, n_streams=None):
        self.LF, self.torch, self.device_io = LF, torch, device_io
        dev = torch.device("cuda:0")
        self.items = []
        for arrs in frames:
            spec, views, sp, mu, beta = arrs
            flags = (LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE) if device_io else 0
            ins = _to_dev(torch, arrs, dev) if device_io else (views, sp, mu)
            self.items.append((spec, _params(LF, spec, beta, storage, "soft", flags), ins))
        # the server's streams do not wait for torch's: the input copies are
        # complete before any frame is submitted
        torch.cuda.synchronize()
        self.ring = ring
        self.rings = {}

    def preallocate(self, stream, spec):
        """Allocates the stream's whole ring of output buffers, so that no
        allocation (which can wait for the device) falls in a timed region."""
        for seq in range(self.ring):
            self.outputs(stream, spec, seq)
        if self.device_io:
            self.torch.cuda.synchronize()

    def outputs(self, stream, spec, seq):
        key = (stream, seq % self.ring)
        o = self.rings.get(key)
        if o is None or o[0] != (spec.H, spec.W):
            if self.device_io:
                dev = self.torch.device("cuda:0")
                o = ((spec.H, spec.W), self.torch.empty((spec.H, spec.W, 3), dtype=self.torch.float32, device=dev),
                     self.torch.empty((spec.H, spec.W), dtype=self.torch.int32, device=dev))
            else:
                o = ((spec.H, spec.W), np.empty((spec.H, spec.W, 3), np.float32), np.empty((spec.H, spec.W), np.int32))
            self.rings[key] = o
        return o[1], o[2]


class Driver:
    """Submits frames and collects completions.  A stream's frame n reuses the
    output buffers of its frame n - ring, so it waits for that one first."""

    def __init__(self, LF, srv, frames: Frames):
        import queue
        self.LF, self.srv, self.frames = LF, srv, frames
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.done_ids = set()
        self.statuses = {}
        self.seq = {}
        self.fids = {}
        self.completed = 0
        self.q = queue.Queue()
        self._cb = LF.lf_done_fn(self._on_done)

    def _on_done(self, fid, status, user):
        with self.cv:
            self.done_ids.add(fid)
            self.statuses[fid] = status
            self.completed += 1
            self.cv.notify_all()
        self.q.put(fid)

    def submit(self, stream, idx):
        spec, p, ins = self.frames.items[idx]
        n = self.seq.get(stream, 0)
        self.seq[stream] = n + 1
        prev = self.fids.get((stream, n - self.frames.ring))
        if prev is not None:
            with self.cv:
                self.cv.wait_for(lambda: prev in self.done_ids, timeout=60.0)
        rgb, d = self.frames.outputs(stream, spec, n)
        while True:
            try:
                fid = self.LF.lf_submit_frame(self.srv, stream, p, *ins, rgb, d, None, self._cb)
                break
            except self.LF.LFError as e:
                if e.status != self.LF.LF_EAGAIN:
                    raise
                time.sleep(0.0002)
        self.fids[(stream, n)] = fid
        return fid

    def wait_count(self, n, timeout=120.0):
        with self.cv:
            ok = self.cv.wait_for(lambda: self.completed >= n, timeout=timeout)
        assert ok, f"{self.completed} of {n} frames completed"

    def check(self):
        bad = {k: v for k, v in self.statuses.items() if v != 0}
        assert not bad, bad


def _stats_dict(st, wall, frames, units):
    return {"frames_per_s": frames / wall, "gunits_per_s": units / wall / 1e9, "p50_ms": st.p50_ms,
            "p99_ms": st.p99_ms, "mean_batch_frames": st.mean_batch_frames,
            "max_batch_frames": int(st.max_batch_frames), "frames": int(st.completed),
            "hbm_peak_bytes": int(st.hbm_peak)}


def _units(spec):
    return spec.H * spec.W * spec.D * spec.K * spec.n_iters


def closed_loop(LF, srv, drv, stream_frames, per_stream, outstanding=2):
    """Every stream keeps `outstanding` frames in flight until it has sent
    per_stream frames.  stream_frames[s] lists the frame indices stream s
    cycles through.  Returns (wall seconds, frames, units)."""
    n_streams = len(stream_frames)
    LF.lf_server_reset_stats(srv)
    base = drv.completed
    sent = [0] * n_streams
    by_fid = {}
    t0 = time.perf_counter()
    for s in range(n_streams):
        for _ in range(outstanding):
            idx = stream_frames[s][sent[s] % len(stream_frames[s])]
            by_fid[drv.submit(s, idx)] = s
            sent[s] += 1
    total = n_streams * per_stream
    units, done = 0, 0
    while done < total:
        fid = drv.q.get(timeout=120.0)
        s = by_fid.pop(fid)
        done += 1
        units += _units(drv.frames.items[stream_frames[s][0]][0])
        if sent[s] < per_stream:
            idx = stream_frames[s][sent[s] % len(stream_frames[s])]
            by_fid[drv.submit(s, idx)] = s
            sent[s] += 1
    return time.perf_counter() - t0, total, units


def one_at_a_time(LF, srv, drv, idx, n):
    """n frames of one stream, each submitted after the previous completed:
    the server's latency on an idle GPU."""
    LF.lf_server_reset_stats(srv)
    for _ in range(n):
        fid = drv.submit(0, idx)
        while drv.q.get(timeout=60.0) != fid:
            pass
    return LF.lf_server_stats(srv)


def drain_queue(drv):
    import queue
    while True:
        try:
            drv.q.get_nowait()
        except queue.Empty:
            return


def _serving_switch_interval():
    """The frame server calls back into Python from its worker threads; with
    the interpreter's default 5 ms switch interval a callback can wait that
    long for the GIL while the submitting thread runs, which is the driver's
    delay, not the server's."""
    sys.setswitchinterval(1e-4)


def serve_same_workload(args, LF, torch, arrs, n_streams=8, per_stream=100, outstanding=2):
    """The headline frame through the FP16 frame server with device-resident
    inputs and outputs: saturation frames/s with n_streams camera streams in
    a closed loop (`outstanding` frames in flight per stream, so that the
    host's submission of the next frame stays off the critical path), and
    single-frame latency on an idle GPU."""
    spec = arrs[0]
    frames = Frames(LF, torch, [arrs], "f16", device_io=True)
    srv = LF.lf_server_create(2 << 30, n_streams, spec.n_iters, 64 << 20)
    drv = Driver(LF, srv, frames)
    try:
        for s in range(n_streams):                      # warm-up: one frame per stream
            frames.preallocate(s, spec)
            drv.submit(s, 0)
        LF.lf_server_drain(srv)
        drain_queue(drv)
        idle = one_at_a_time(LF, srv, drv, 0, max(args.latency_frames, 100))
        drain_queue(drv)
        wall, n, units = closed_loop(LF, srv, drv, [[0]] * n_streams, per_stream, outstanding)
        LF.lf_server_drain(srv)
        sat = LF.lf_server_stats(srv)
        drv.check()
    finally:
        LF.lf_server_destroy(srv)
    return {"storage": "f16", "io": "device", "camera_streams": n_streams, "outstanding_per_stream": outstanding,
            "saturation": _stats_dict(sat, wall, n, units),
            "single_frame_latency": {"p50_ms": idle.p50_ms, "p99_ms": idle.p99_ms, "frames": int(idle.completed)}}


def serve_mix(args, LF, torch, mix, device_io, poisson_levels=(0.3, 0.5, 0.7, 0.9), budget=1 << 30):
    """The 16-stream serving mix (two frames per stream, alternating) through
    the FP16 frame server: saturation in a closed loop, then Poisson arrivals
    over the 16 streams at fractions of the saturation rate."""
    import random
    frames = Frames(LF, torch, mix, "f16", device_io=device_io)
    n_iters = mix[0][0].n_iters
    srv = LF.lf_server_create(budget, SERVE_STREAMS, n_iters, 1 << 30)
    drv = Driver(LF, srv, frames)
    stream_frames = [[2 * s, 2 * s + 1] for s in range(SERVE_STREAMS)]
    out = {"workload": "serving-mix-fp16-i8: 16 streams, 320x240/640x480/1280x960 (5/8/3 streams), K 3/5/7, "
                       "D 32/64/128, objects moving 2 px/frame, warm start per stream",
           "io": "device" if device_io else "host (PCIe copies included)", "hbm_budget_bytes": budget}
    try:
        for s in range(SERVE_STREAMS):                  # warm-up: one frame per stream
            frames.preallocate(s, frames.items[2 * s][0])
            drv.submit(s, 2 * s)
        LF.lf_server_drain(srv)
        drain_queue(drv)
        wall, n, units = closed_loop(LF, srv, drv, stream_frames, 24 if device_io else 12)
        LF.lf_server_drain(srv)
        drain_queue(drv)
        sat = LF.lf_server_stats(srv)
        out["saturation"] = _stats_dict(sat, wall, n, units)
        fps_sat = n / wall
        log(args, f"serving mix ({out['io']}): saturation {fps_sat:.0f} frames/s, p99 {sat.p99_ms:.2f} ms")
        rng = random.Random(7)
        for level in (poisson_levels if device_io else ()):
            rate = level * fps_sat
            n_frames = max(args.poisson_frames, 200)
            LF.lf_server_reset_stats(srv)
            base = drv.completed
            t, units = 0.0, 0
            t0 = time.perf_counter()
            for i in range(n_frames):
                t += rng.expovariate(rate)
                s = rng.randrange(SERVE_STREAMS)
                idx = stream_frames[s][drv.seq.get(s, 0) % 2]
                units += _units(frames.items[idx][0])
                delay = t0 + t - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                drv.submit(s, idx)
            drv.wait_count(base + n_frames)
            wall = time.perf_counter() - t0
            st = LF.lf_server_stats(srv)
            drain_queue(drv)
            d = _stats_dict(st, wall, n_frames, units)
            d["offered_frames_per_s"] = rate
            out[f"poisson_{level}"] = d
            log(args, f"serving mix poisson {level}: {d['frames_per_s']:.0f} frames/s, p50 {st.p50_ms:.2f} ms, "
                      f"p99 {st.p99_ms:.2f} ms")
        drv.check()
    finally:
        LF.lf_server_destroy(srv)
    return out


def large_concurrent(args, LF, torch, large, reps=5):
    """Four large-workload streams (BF16) submitted together and run in one
    server launch, beside the plain FP32 context on the same four frames."""
    spec = large[0][0]
    frames = Frames(LF, torch, large, "bf16", device_io=True, ring=2)
    n = len(large)
    for s in range(n):
        frames.preallocate(s, spec)
    srv = LF.lf_server_create(4 << 30, n, spec.n_iters, 64 << 20)
    drv = Driver(LF, srv, frames)
    try:
        walls = []
        for r in range(reps + 1):
            LF.lf_server_hold(srv, 1)                   # queue the four, then release them together
            for s in range(n):
                drv.submit(s, s)
            if r == 1:
                LF.lf_server_reset_stats(srv)
            t0 = time.perf_counter()
            LF.lf_server_hold(srv, 0)
            LF.lf_server_drain(srv)
            if r >= 1:
                walls.append(time.perf_counter() - t0)
        st = LF.lf_server_stats(srv)
        drv.check()
    finally:
        LF.lf_server_destroy(srv)
    wall = float(np.median(walls))
    served = {"storage": "bf16", "streams": n, "frames_per_launch": st.mean_batch_frames,
              "max_batch_frames": int(st.max_batch_frames), "ms_per_group": wall * 1e3,
              "frames_per_s": n / wall, "gunits_per_s": n * _units(spec) / wall / 1e9,
              "p50_ms": st.p50_ms, "p99_ms": st.p99_ms}
    # the plain FP32 context on the same frames, one frame after the other
    dev = torch.device("cuda:0")
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE | LF.LF_DEFERRED_CHECK
    ins = [_to_dev(torch, a, dev) for a in large]
    p = _params(LF, spec, large[0][4], "f32", "soft", flags)
    K, H, W = spec.K, spec.H, spec.W
    out = (torch.empty((H, W, 3), device=dev), torch.empty((H, W), dtype=torch.int32, device=dev),
           torch.empty((K, H, W), device=dev), torch.empty((H, W), dtype=torch.uint8, device=dev))
    ctx = LF.lf_em_init(p, *ins[0], hip_stream=torch.cuda.current_stream().cuda_stream)
    try:
        walls = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                LF.lf_em_load(ctx, *ins[i])
                LF.lf_em_iterate(ctx, spec.n_iters)
                LF.lf_refocus(ctx, *out, 0)
            torch.cuda.synchronize()
            if r >= 1:
                walls.append(time.perf_counter() - t0)
        LF.lf_em_check(ctx)
    finally:
        LF.lf_em_destroy(ctx)
    wall_p = float(np.median(walls))
    plain = {"storage": "f32", "frames_per_s": n / wall_p, "gunits_per_s": n * _units(spec) / wall_p / 1e9,
             "ms_per_frame": wall_p / n * 1e3}
    return {"workload": spec.name, "server_one_launch_bf16": served, "plain_context_fp32": plain,
            "parity": "server frames equal the plain context's bits at the same storage (tests/test_gpu_server.py); "
                      "BF16 and FP32 each match the oracle with their own storage on sampled rows "
                      "(tests/test_gpu_parity.py, tests/test_gpu_configs.py)"}


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host cores
# ---------------------------------------------------------------------------

def _host_cpu():
    model, cores = platform.processor() or "unknown", set()
    try:
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, (len(cores) or None), avail


def _oracle_params(O, spec, beta, storage, mode):
    return O.make_params(spec.K, spec.H, spec.W, spec.ref, [float(np.float32(b)) for b in spec.baselines],
                         float(np.float32(spec.d_min)), float(np.float32(spec.d_step)), spec.D,
                         float(np.float32(beta)), float("nan"), float(np.float32(spec.gamma)),
                         float(np.float32(spec.sigma)), float(np.float32(spec.tau)), storage, mode)


_ONE_CORE = r"""
import sys, time, json
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as O
d = np.load(sys.argv[2])
p = O.make_params(*json.loads(sys.argv[3]))
rows = (0, int(sys.argv[4]))
t0 = time.perf_counter()
r = O.reconstruct(p, d["views"], d["S_P"], d["mu_T"], int(sys.argv[5]), rows=rows)
print(json.dumps({"seconds": time.perf_counter() - t0, "threads": int(r["threads"])}))
"""


def cpu_baseline(args, arrs, storage, mode, budget_s):
    """The FP64 oracle as it stands on the host: whole frames of the same
    workload with every host thread (median of three runs, each about a third
    of the budget), and a band of rows with one thread (a child process)."""
    import tempfile
    import oracle as O
    spec, views, sp, mu, beta = arrs
    p = _oracle_params(O, spec, beta, storage, mode)
    O.lib()
    units_frame = spec.H * spec.W * spec.D * spec.K * spec.n_iters
    rates, threads, frames_total, el_total = [], 0, 0, 0.0
    for run in range(3):
        frames, t0 = 0, time.perf_counter()
        while True:
            r = O.reconstruct(p, views, sp, mu, spec.n_iters)
            frames += 1
            el = time.perf_counter() - t0
            if el >= budget_s / 3 or frames >= 20:
                break
        rates.append(units_frame * frames / el / 1e9)
        threads = int(r["threads"])
        frames_total += frames
        el_total += el
    model, phys, avail = _host_cpu()
    # one thread on a band of rows
    band = max(8, min(spec.H, spec.H // 10))
    one = None
    try:
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "frame.npz")
            np.savez(path, views=views, S_P=sp, mu_T=mu)
            pargs = [spec.K, spec.H, spec.W, spec.ref, [float(np.float32(b)) for b in spec.baselines],
                     float(np.float32(spec.d_min)), float(np.float32(spec.d_step)), spec.D,
                     float(np.float32(beta)), float("nan"), float(np.float32(spec.gamma)),
                     float(np.float32(spec.sigma)), float(np.float32(spec.tau)), storage, mode]
            env = dict(os.environ, OMP_NUM_THREADS="1")
            res = subprocess.run([sys.executable, "-c", _ONE_CORE, ROOT, path, json.dumps(pargs), str(band),
                                  str(spec.n_iters)], capture_output=True, text=True, env=env, timeout=300)
            rec = json.loads(res.stdout.strip().splitlines()[-1])
            one = {"value": spec.W * band * spec.D * spec.K * spec.n_iters / rec["seconds"] / 1e9,
                   "threads": rec["threads"], "sample": f"rows 0-{band} of one frame, {rec['seconds']:.1f} s"}
    except Exception as e:      # the one-thread figure is context only
        one = {"error": str(e)[:200]}
    return {"value": float(np.median(rates)), "unit": "EM-iter Gpix·disp·view/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{frames_total} full frame(s) of the same workload over 3 runs ({el_total:.1f} s), "
                      f"median of the runs, FP64 C/OpenMP",
            "runs": rates, "frames_per_s": float(np.median(rates)) * 1e9 / units_frame,
            "host": {"cpu_model": model, "physical_cores": phys, "cpus_available": avail},
            "one_thread": one}


# ---------------------------------------------------------------------------

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "the per-GPU work shards by row bands, see the design notes.", file=sys.stderr)
        sys.exit(2)
    inputs = make_inputs(args)
    import torch
    import paper_2003_11076_amd as LF

    main_arrs = inputs["main"][0]
    spec = main_arrs[0]
    storage = args.storage or spec.storage
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calib_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the
        # counters read for the EM kernel
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n_streams = max(1, args.streams)
    log(args, f"{spec.name}: warmup {args.warmup}, timing {args.steps} steps over {n_streams} stream(s)")
    m = form_leg(args, LF, torch, main_arrs, storage, args.steps, args.warmup, n_streams, args.mode)
    out = {
        "metric": "EM-iter Gpix·disp·view/s",
        "value": m["value"],
        "unit": "EM-iter Gpix·disp·view/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene generator, uint8 views, float32 S_P and mu_T)",
        "config": {"workload": spec.name, "K": spec.K, "H": spec.H, "W": spec.W, "D": spec.D,
                   "em_iters": spec.n_iters, "storage": storage, "mode": args.mode, "parallelism": "single-gpu",
                   "streams": n_streams},
        "p50_ms": m["p50_ms"],
        "p99_ms": m["p99_ms"],
        "latency_frames": m["latency_frames"],
        "frames_per_s": m["frames_per_s"],
        "em_ms_timed_region": m["em_ms_timed_region"],
        "em_busy_ms_per_step": m["em_busy_ms_per_step"],
        "em_ms_alone": m["em_ms_alone"],
        "roofline": m["roofline"],
    }
    if not args.no_forms:
        out["forms"] = {}
        for name, st in (("precision", "f16"), ("large", "bf16")):
            arrs = inputs[name][0]
            steps = max(10, args.steps // (2 if name == "precision" else 10))
            log(args, f"{arrs[0].name}: timing {steps} steps")
            out["forms"][name] = form_leg(args, LF, torch, arrs, st, steps, max(2, args.warmup // 4), n_streams)
    if not args.no_variants:
        log(args, "timing the variants (search window, dynamic-only, enumeration)")
        out["variants"] = variant_legs(LF, torch, main_arrs, storage)
        if "precision" in inputs:
            out["variants"]["dynamic_only_precision"] = variant_legs(
                LF, torch, inputs["precision"][0], "f16", reps=10, names=("plain", "dynamic_only"))
    if not args.no_serving:
        _serving_switch_interval()
        log(args, "serving the headline frame through the FP16 frame server (device buffers)")
        sw = serve_same_workload(args, LF, torch, main_arrs)
        sw["vs_plain_fp32"] = {"frames_per_s_ratio": sw["saturation"]["frames_per_s"] / m["frames_per_s"],
                               "plain_frames_per_s": m["frames_per_s"], "plain_p99_ms": m["p99_ms"],
                               "plain_p50_ms": m["p50_ms"]}
        out["serving_same_workload"] = sw
        log(args, f"serving same workload: {sw['saturation']['frames_per_s']:.0f} frames/s "
                  f"(plain {m['frames_per_s']:.0f}); single-frame p99 {sw['single_frame_latency']['p99_ms']:.3f} ms "
                  f"(plain {m['p99_ms']:.3f})")
        out["serving"] = serve_mix(args, LF, torch, inputs["mix"], device_io=True)
        out["serving_host_io"] = serve_mix(args, LF, torch, inputs["mix"], device_io=False)
    if not args.no_forms:
        log(args, "four large streams in one server launch, and the plain FP32 context on the same frames")
        out["large_concurrent"] = large_concurrent(args, LF, torch, inputs["large"])
    if not args.no_cpu_baseline:
        log(args, "timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args, main_arrs, storage, args.mode, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
