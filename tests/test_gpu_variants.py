"""Work-avoiding variants through the C ABI: the M-step window around mu_T
(LF_PRIOR_WINDOW, Sec. III-C) and reconstruction of the dynamic reference
pixels only (LF_DYNAMIC_ONLY, Sec. III-F / IV-B).  Parity against the FP64
oracle run with the same variant, plus bitwise relations to the plain path."""
import sys

import numpy as np
import pytest

import lf_scenes as S
from lfcase import Case, DeviceRun, random_case, teacher_forced

pytestmark = pytest.mark.gpu

WINDOW, DYN = 0x8, 0x10


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("flags", [WINDOW, DYN, WINDOW | DYN])
@pytest.mark.parametrize("mode", ["soft", "hard"])
def test_small_scene_variants_teacher_forced(flags, mode):
    case = Case.from_frame(S.make_frame(S.workload_spec("small")), storage="f32", mode=mode, flags=flags)
    _say(f"small_frame 160x120 K=5 D=32 fp32 {mode} flags={flags:#x} teacher-forced x3")
    teacher_forced(case, 3)


SMALL = [
    # K, H, W, D, baselines, d_min, d_step, storage
    (3, 5, 300, 24, [-1, 0, 2], -2, 1, "f16"),
    (5, 4, 129, 40, None, 0, 1, "bf16"),
    (4, 3, 70, 16, [-1.5, 0, 0.5, 2.25], 0, 0.5, "f32"),   # fractional shifts
    (9, 2, 200, 48, None, 0, 1, "f32"),
    (7, 2, 257, 33, None, 3, 2, "f16"),
]


@pytest.mark.parametrize("K,H,W,D,b,dmin,dstep,st", SMALL)
@pytest.mark.parametrize("flags", [WINDOW, DYN | WINDOW])
def test_small_variants_teacher_forced(K, H, W, D, b, dmin, dstep, st, flags):
    case = random_case(K, H, W, D, baselines=b, d_min=dmin, d_step=dstep, storage=st, seed=K * 100 + W)
    case.flags = flags
    _say(f"variants small K={K} H={H} W={W} D={D} b={b} d=({dmin},{dstep}) {st} flags={flags:#x}")
    teacher_forced(case, 3)


def test_large_window_sampled_rows():
    case = Case.from_frame(S.make_frame(S.workload_spec("large")), storage="bf16", flags=WINDOW | DYN)
    _say("large 1920x1080 K=9 D=192 bf16 window+dynamic-only teacher-forced x4, rows 530..538")
    teacher_forced(case, 4, rows=(530, 538))


def _run(case, flags, n=3):
    run = DeviceRun(case, extra_flags=flags)
    run.iterate(n)
    out = run.refocus()
    L = run.state()[2]
    run.close()
    return out, L


def test_dynamic_only_equals_plain_on_dynamic_pixels():
    case = Case.from_frame(S.make_frame(S.workload_spec("small")), storage="f32")
    _say("small_frame dynamic-only vs plain, bitwise on the dynamic reference pixels")
    (rgb0, d0, q0, h0), L0 = _run(case, 0)
    (rgb1, d1, q1, h1), L1 = _run(case, DYN)
    run = DeviceRun(case)
    _, rho = run.intermediates()
    run.close()
    dyn = rho[case.ref] < np.float32(case.tau)
    assert dyn.any() and (~dyn).any()
    assert np.array_equal(d1[dyn], d0[dyn]) and np.array_equal(q1[:, dyn], q0[:, dyn])
    assert np.array_equal(rgb1[dyn], rgb0[dyn]) and np.array_equal(h1[dyn], h0[dyn])
    assert np.array_equal(L1[dyn], L0[dyn]) and np.all(L1[~dyn] == 0)
    assert np.array_equal(rgb1[~dyn], case.views[case.ref][~dyn].astype(np.float32) / np.float32(255))
    assert not h1[~dyn].any()


def test_dynamic_only_work_list_shapes():
    """Rows whose dynamic pixels cut into work items in every way: a whole
    dynamic row (items of 64), pixels 100 columns apart (items closed by the
    span), a dense run then a lone pixel in the last column, one dynamic pixel
    at column 0, no dynamic pixel.  Bitwise equal to the plain path on the
    dynamic pixels, level nearest mu_T and objective 0 on the others; and the
    oracle's dynamic-only run, teacher-forced."""
    case = random_case(5, 5, 600, 24, storage="f16", seed=41)
    tau = float(case.tau)
    sp = case.S_P.copy()
    ref = case.ref
    sp[ref] = np.float32(min(tau + 0.2, 1.0))
    sp[ref, 0, :] = 0.1
    sp[ref, 1, ::100] = 0.1
    sp[ref, 2, 150:350] = 0.1
    sp[ref, 2, -1] = 0.1
    sp[ref, 3, 0] = 0.1
    case.S_P = sp
    _say("dynamic-only work list shapes 600x5 K=5 D=24 f16")
    (rgb0, d0, q0, h0), L0 = _run(case, 0)
    (rgb1, d1, q1, h1), L1 = _run(case, DYN)
    run = DeviceRun(case)
    _, rho = run.intermediates()
    run.close()
    dyn = rho[ref] < np.float32(case.tau)
    assert dyn[0].all() and dyn[1].sum() == 6 and dyn[2].sum() == 201 and dyn[3].sum() == 1 and not dyn[4].any()
    assert np.array_equal(d1[dyn], d0[dyn]) and np.array_equal(q1[:, dyn], q0[:, dyn])
    assert np.array_equal(L1[dyn], L0[dyn]) and np.all(L1[~dyn] == 0)
    d_min, d_step = float(case.d_min), float(case.d_step)
    near = np.clip(np.ceil((case.mu_T.astype(np.float64) - d_min) / d_step - 0.5), 0, case.D - 1).astype(np.int32)
    assert np.array_equal(d1[~dyn], near[~dyn])
    case.flags = DYN
    teacher_forced(case, 3)


@pytest.mark.parametrize("cover", ["none", "all"])
def test_dynamic_only_with_no_or_every_pixel_dynamic(cover):
    """No dynamic reference pixel: an empty work list (every EM block exits),
    every pixel at the level nearest mu_T with objective 0 and its reference
    colour.  Every pixel dynamic: the plain path's bits everywhere."""
    case = random_case(5, 6, 300, 24, storage="bf16", seed=43)
    sp = case.S_P.copy()
    sp[case.ref] = np.float32(0.95) if cover == "none" else np.float32(0.05)
    case.S_P = sp
    _say(f"dynamic-only with {cover} of the reference pixels dynamic, 300x6 K=5 D=24 bf16")
    (rgb0, d0, q0, h0), L0 = _run(case, 0)
    (rgb1, d1, q1, h1), L1 = _run(case, DYN)
    if cover == "all":
        for a, b in ((rgb0, rgb1), (d0, d1), (q0, q1), (h0, h1), (L0, L1)):
            assert np.array_equal(a, b)
    else:
        d_min, d_step = float(case.d_min), float(case.d_step)
        near = np.clip(np.ceil((case.mu_T.astype(np.float64) - d_min) / d_step - 0.5), 0, case.D - 1)
        assert np.array_equal(d1, near.astype(np.int32)) and np.all(L1 == 0) and not h1.any()
        assert np.array_equal(rgb1, case.views[case.ref].astype(np.float32) / np.float32(255))


def test_window_covering_all_levels_is_the_plain_sweep():
    """With 3 sigma wider than the level range the window holds every level:
    same bits as the plain sweep (fast and exhaustive)."""
    import paper_2003_11076_amd as LF
    case = random_case(5, 6, 200, 24, storage="f16", seed=9)
    case.sigma = np.float32(20.0)
    _say("window wider than the level range vs plain sweep, fast and exhaustive")
    for extra in (0, LF.LF_EXHAUSTIVE_SWEEP):
        (a, La) = _run(case, extra)
        (b, Lb) = _run(case, WINDOW | extra)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.array_equal(La, Lb)


def test_window_fast_sweep_matches_exhaustive():
    import paper_2003_11076_amd as LF
    case = random_case(7, 4, 300, 64, storage="bf16", seed=10)
    _say("window: fast vs exhaustive sweep K=7 4x300 D=64 bf16")
    (a, La) = _run(case, WINDOW | DYN)
    (b, Lb) = _run(case, WINDOW | DYN | LF.LF_EXHAUSTIVE_SWEEP)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(La, Lb)


SERVER_CASES = [
    dict(K=5, H=6, W=260, D=40, storage="f16", flags=WINDOW | DYN),
    dict(K=7, H=4, W=140, D=24, storage="f32", flags=DYN, mode="enum_soft"),
    dict(K=3, H=5, W=90, D=16, storage="bf16", flags=WINDOW, mode="hard"),
]


@pytest.mark.parametrize("kw", SERVER_CASES)
def test_server_variants_equal_plain_context(kw):
    from test_gpu_server import Server, _plain
    kw = dict(kw)
    flags = kw.pop("flags")
    case = random_case(kw.pop("K"), kw.pop("H"), kw.pop("W"), kw.pop("D"), seed=12, **kw)
    case.flags = flags
    _say(f"server vs plain context with flags={flags:#x} K={case.K} {case.storage} {case.mode}")
    with Server(n_iters=3) as srv:
        fid, (rgb, d, q) = srv.submit(0, case)
        srv.drain()
        assert srv.done == {fid: 0}
    prgb, pd, pq = _plain(case, 3)
    assert np.array_equal(d, pd) and np.array_equal(q, pq) and np.array_equal(rgb, prgb)
