"""Two contexts on two HIP streams with frames dealt round robin, as
bench.py's throughput loop deals them: every frame's outputs are the same
bits as the same frame processed alone, one at a time."""
import sys

import numpy as np
import pytest

import lf_scenes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_two_streams_give_the_bits_of_one():
    import torch
    import paper_2003_11076_amd as LF
    dev = torch.device("cuda:0")
    frames = []
    for shift in (0.0, 1.0, -0.5, 2.0):
        fr = S.make_frame(S.workload_spec("small"))
        frames.append((fr, (fr.mu_T + np.float32(shift)).astype(np.float32)))
    sp = frames[0][0].spec
    K, H, W = sp.K, sp.H, sp.W
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE | LF.LF_DEFERRED_CHECK
    p = LF.make_params(K, H, W, sp.ref, sp.baselines, sp.d_min, sp.d_step, sp.D, frames[0][0].beta,
                       gamma=sp.gamma, sigma=sp.sigma, tau_init=sp.tau, storage="f32", flags=flags)
    ins = [(torch.from_numpy(fr.views).to(dev), torch.from_numpy(fr.S_P).to(dev), torch.from_numpy(mu).to(dev))
           for fr, mu in frames]

    def outputs():
        return (torch.empty((H, W, 3), dtype=torch.float32, device=dev),
                torch.empty((H, W), dtype=torch.int32, device=dev),
                torch.empty((K, H, W), dtype=torch.float32, device=dev),
                torch.empty((H, W), dtype=torch.uint8, device=dev))

    _say(f"small {W}x{H}: {len(frames)} frames alone, then dealt to two streams")
    alone = []
    ctx = LF.lf_em_init(p, *ins[0], hip_stream=torch.cuda.current_stream().cuda_stream)
    for v, s, m in ins:
        out = outputs()
        LF.lf_em_load(ctx, v, s, m)
        LF.lf_em_iterate(ctx, sp.n_iters)
        LF.lf_refocus(ctx, *out, 0)
        torch.cuda.synchronize()
        alone.append([t.cpu().numpy() for t in out])
    LF.lf_em_check(ctx)
    LF.lf_em_destroy(ctx)

    streams = [torch.cuda.Stream(device=dev) for _ in range(2)]
    ctxs = [LF.lf_em_init(p, *ins[0], hip_stream=st.cuda_stream) for st in streams]
    outs = []
    for rep in range(2):
        for i, (v, s, m) in enumerate(ins):
            c = ctxs[(rep * len(ins) + i) % 2]
            out = outputs()
            LF.lf_em_load(c, v, s, m)
            LF.lf_em_iterate(c, sp.n_iters)
            LF.lf_refocus(c, *out, 0)
            outs.append((i, out))
    torch.cuda.synchronize()
    for c in ctxs:
        LF.lf_em_check(c)
        LF.lf_em_destroy(c)
    for i, out in outs:
        for a, b in zip(alone[i], [t.cpu().numpy() for t in out]):
            assert np.array_equal(a, b), i
