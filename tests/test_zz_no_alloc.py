"""The allocation-free whole-frame entry point (lf_em_frame_noalloc) against
the context path it stands in for (lf_em_init, lf_em_iterate with the
objective, lf_refocus, all on the same device inputs): the same bits for the
image, holes, levels, weights and objective, on two calls in a row, the
second on a smaller frame and with the median, so that the second call runs
over what the first left in the scratch array."""
import sys

import numpy as np
import pytest

import lf_scenes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _inputs(spec, dev):
    import torch
    fr = S.make_frame(spec)
    return fr, tuple(torch.from_numpy(a).to(dev) for a in (fr.views, fr.S_P, fr.mu_T))


def _params(LF, fr, flags):
    sp = fr.spec
    return LF.make_params(sp.K, sp.H, sp.W, sp.ref, sp.baselines, sp.d_min, sp.d_step, sp.D, fr.beta,
                          gamma=sp.gamma, sigma=sp.sigma, tau_init=sp.tau, storage=sp.storage, flags=flags)


def _outputs(torch, sp, dev):
    return {"rgb": torch.full((sp.H, sp.W, 3), -1.0, dtype=torch.float32, device=dev),
            "d": torch.full((sp.H, sp.W), -1, dtype=torch.int32, device=dev),
            "q": torch.full((sp.K, sp.H, sp.W), -1.0, dtype=torch.float32, device=dev),
            "hole": torch.full((sp.H, sp.W), 7, dtype=torch.uint8, device=dev)}


def _context_path(LF, torch, fr, ins, n_iters, median, dev, extra=0):
    p = _params(LF, fr, LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE | extra)
    out = _outputs(torch, fr.spec, dev)
    obj = np.zeros(n_iters)
    ctx = LF.lf_em_init(p, *ins, hip_stream=torch.cuda.current_stream().cuda_stream)
    try:
        LF.lf_em_iterate(ctx, n_iters, obj)
        LF.lf_refocus(ctx, out["rgb"], out["d"], out["q"], out["hole"], median)
        torch.cuda.synchronize()
    finally:
        LF.lf_em_destroy(ctx)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["obj"] = obj
    return res


def _noalloc_path(LF, torch, fr, ins, n_iters, median, dev, extra=0):
    p = _params(LF, fr, extra)
    out = _outputs(torch, fr.spec, dev)
    obj = torch.full((n_iters,), -1.0, dtype=torch.float64, device=dev)
    bad = torch.full((1,), 99, dtype=torch.int32, device=dev)
    LF.lf_em_frame_noalloc(p, *ins, None, n_iters, out["rgb"], out["d"], out["q"], out["hole"], median, obj, bad,
                           hip_stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["obj"] = obj.cpu().numpy()
    res["bad"] = int(bad.cpu().item())
    return res


def test_noalloc_gives_the_bits_of_the_context_path_on_two_calls():
    import torch
    import paper_2003_11076_amd as LF
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # the second frame is smaller, with the median; then both again with
    # dynamic-only (its work list lives in the scratch array too)
    dyn = LF.LF_DYNAMIC_ONLY
    cases = [("plain", 0, 0), ("small", 3, 0), ("plain", 0, dyn), ("small", 3, dyn)]
    for name, median, extra in cases:
        spec = S.workload_spec(name)
        fr, ins = _inputs(spec, dev)
        _say(f"noalloc {spec.name} {spec.W}x{spec.H} K={spec.K} D={spec.D} I={spec.n_iters} median={median} "
             f"flags={extra:#x}")
        ref = _context_path(LF, torch, fr, ins, spec.n_iters, median, dev, extra)
        got = _noalloc_path(LF, torch, fr, ins, spec.n_iters, median, dev, extra)
        assert got["bad"] == 0, got["bad"]
        for k in ("rgb", "d", "q", "hole", "obj"):
            assert np.array_equal(ref[k], got[k]), (name, k)


def test_noalloc_rejects_a_frame_beyond_its_scratch():
    import torch
    import paper_2003_11076_amd as LF
    dev = torch.device("cuda:0")
    K, H, W = 9, 1080, 1920
    p = LF.make_params(K, H, W, 4, [k - 4 for k in range(K)], 0, 1, 192, 2000.0)
    _say(f"noalloc size check {W}x{H} K={K}")
    tiny = torch.zeros(16, dtype=torch.float32, device=dev)
    with pytest.raises(LF.LFError) as e:
        LF.lf_em_frame_noalloc(p, tiny, tiny, tiny, None, 1, tiny, tiny, tiny)
    assert e.value.status == LF.LF_EINVAL and "scratch" in str(e.value)
