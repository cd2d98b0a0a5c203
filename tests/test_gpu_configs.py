"""Parity at the configurations the benchmark times.

* Serving mix at full size: for each of the 16 stream shapes (three sizes,
  K in {3, 5, 7}, D in {32, 64, 128}, FP16), two consecutive frames of the
  stream go through the frame server in one run (the second warm-started
  from the first).  The second frame is then run by the plain context from
  the server's first-frame weights, one iteration at a time against the FP64
  oracle on four bands of rows (top, bottom, through a moving object,
  middle), and the server's outputs must equal that chain's final state bit
  for bit on the whole frame.
* The headline frame in the benchmark's launch configuration (two contexts
  on two HIP streams, all iterations in one launch, deferred input check,
  device outputs) gives the bits of the one-iteration-at-a-time chain that
  the full-frame teacher-forced test checks against the oracle.
* Device outputs equal host outputs, with the median and with dynamic-only.
"""
import multiprocessing as mp
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import lf_scenes as S
from lfcase import Case, DeviceRun, teacher_forced, row_bands, workload_frame

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _generate(specs):
    # fresh interpreters (spawn): this process has initialised the GPU runtime
    with ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(S.frame_arrays, specs))


def test_serving_mix_shapes_against_the_oracle():
    import threading
    import torch
    import paper_2003_11076_amd as LF
    n_streams = 16
    specs = [S.serving_stream_spec(s, f) for s in range(n_streams) for f in range(2)]
    _say(f"serving mix: generating {len(specs)} frames of {n_streams} stream shapes")
    arrs = _generate(specs)
    dev = torch.device("cuda:0")
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE
    lock, status = threading.Lock(), {}

    def on_done(fid, st, user):
        with lock:
            status[fid] = st

    cb = LF.lf_done_fn(on_done)
    keep, outs = [], {}
    _say("serving mix: two frames per stream through the server (FP16, 8 iterations, device buffers)")
    srv = LF.lf_server_create(4 << 30, n_streams, 8, 64 << 20)
    try:
        for f in range(2):
            for s in range(n_streams):
                sp = specs[2 * s + f]
                views, S_P, mu, beta = arrs[2 * s + f]
                p = LF.make_params(sp.K, sp.H, sp.W, sp.ref, sp.baselines, sp.d_min, sp.d_step, sp.D, beta,
                                   gamma=sp.gamma, sigma=sp.sigma, tau_init=sp.tau, storage="f16", flags=flags)
                ins = [torch.from_numpy(a).to(dev) for a in (views, S_P, mu)]
                o = (torch.zeros((sp.H, sp.W, 3), device=dev), torch.zeros((sp.H, sp.W), dtype=torch.int32, device=dev),
                     torch.zeros((sp.K, sp.H, sp.W), device=dev))
                keep.append(ins)
                outs[s, f] = o
                # the server's streams do not wait for torch's: the copies and
                # fills above must be done before the frame is submitted
                torch.cuda.synchronize()
                LF.lf_submit_frame(srv, s, p, *ins, *o, cb)
        LF.lf_server_drain(srv)
    finally:
        LF.lf_server_destroy(srv)
    torch.cuda.synchronize()
    assert len(status) == 2 * n_streams and all(v == 0 for v in status.values()), status
    for s in range(n_streams):
        sp = specs[2 * s + 1]
        views, S_P, mu, beta = arrs[2 * s + 1]
        case = Case.from_arrays(sp, views, S_P, mu, beta, storage="f16")
        q1 = outs[s, 0][2].cpu().numpy()
        expect = [t.cpu().numpy() for t in outs[s, 1]]
        for band in row_bands(case):
            _say(f"serving stream {s}: {sp.W}x{sp.H} K={sp.K} D={sp.D} frame 2, rows {band[0]}..{band[1]}")
            teacher_forced(case, 8, rows=band, q_warm=q1, expect=expect)


def test_bench_launch_configuration_gives_the_chain_bits():
    import torch
    import paper_2003_11076_amd as LF
    fr = workload_frame("plain")
    case = Case.from_frame(fr, storage="f32")
    dev = torch.device("cuda:0")
    K, H, W, I = case.K, case.H, case.W, case.n_iters
    _say(f"plain {W}x{H}: one iteration at a time, single context")
    run = DeviceRun(case)
    for _ in range(I):
        run.iterate(1)
    chain = run.refocus()
    run.close()
    _say("plain: the benchmark's configuration (two streams, one launch, deferred check, device outputs)")
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE | LF.LF_DEFERRED_CHECK
    p = case.api_params(flags)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (case.views, case.S_P, case.mu_T)]
    streams = [torch.cuda.current_stream(), torch.cuda.Stream(device=dev)]
    ctxs = [LF.lf_em_init(p, *ins, hip_stream=st.cuda_stream) for st in streams]
    outs = []
    try:
        for i in range(6):
            c = ctxs[i % 2]
            o = (torch.empty((H, W, 3), device=dev), torch.empty((H, W), dtype=torch.int32, device=dev),
                 torch.empty((K, H, W), device=dev), torch.empty((H, W), dtype=torch.uint8, device=dev))
            LF.lf_em_load(c, *ins)
            LF.lf_em_iterate(c, I)
            LF.lf_refocus(c, *o, 0)
            outs.append(o)
        torch.cuda.synchronize()
        for c in ctxs:
            LF.lf_em_check(c)
    finally:
        for c in ctxs:
            LF.lf_em_destroy(c)
    for o in outs:
        for a, b in zip(chain, o):
            assert np.array_equal(a, b.cpu().numpy())


@pytest.mark.parametrize("median,dyn_only", [(0, False), (3, False), (3, True)])
def test_device_outputs_equal_host_outputs(median, dyn_only):
    import torch
    import paper_2003_11076_amd as LF
    fr = workload_frame("small")
    case = Case.from_frame(fr, storage="f32")
    extra = LF.LF_DYNAMIC_ONLY if dyn_only else 0
    _say(f"small: device vs host outputs, median={median} dynamic-only={dyn_only}")
    run = DeviceRun(case, extra_flags=extra)
    run.iterate(case.n_iters)
    host = run.refocus(median)
    run.close()
    dev = torch.device("cuda:0")
    K, H, W = case.K, case.H, case.W
    run = DeviceRun(case, extra_flags=extra | LF.LF_OUTPUTS_ON_DEVICE)
    run.iterate(case.n_iters)
    o = (torch.full((H, W, 3), -1.0, device=dev), torch.full((H, W), -1, dtype=torch.int32, device=dev),
         torch.full((K, H, W), -1.0, device=dev), torch.full((H, W), 7, dtype=torch.uint8, device=dev))
    LF.lf_refocus(run.ctx, *o, median)
    torch.cuda.synchronize()
    run.close()
    for a, b in zip(host, o):
        assert np.array_equal(a, b.cpu().numpy())
