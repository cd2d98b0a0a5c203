"""Parity of the HIP path against the FP64 oracle, through the C ABI.

Each test prints the case it runs (and flushes) before touching the GPU.
Tolerances and exemptions are those of tests/lfcase.py.
"""
import sys

import numpy as np
import pytest

import lf_scenes as S
import oracle as O
from lfcase import Case, DeviceRun, random_case, teacher_forced, near_tie, row_bands, workload_frame

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small_frame():
    return S.make_frame(S.workload_spec("small"))


@pytest.mark.parametrize("mode", ["soft", "hard"])
def test_small_teacher_forced(small_frame, mode):
    case = Case.from_frame(small_frame, storage="f32", mode=mode)
    _say(f"small_frame 160x120 K=5 D=32 fp32 {mode} teacher-forced x5")
    stats = teacher_forced(case, 5)
    assert sum(s.get("near_ties", 0) for s in stats[:-1]) < 0.01 * case.H * case.W * 5


SMALL = [
    # K, H, W, D, baselines, d_min, d_step, storage
    (2, 7, 37, 9, [0, 1], 0, 1, "f32"),                   # W below one tile
    (3, 5, 300, 16, [-1, 0, 2], -2, 1, "f16"),            # ragged last tile, negative levels
    (5, 4, 129, 24, None, 0, 1, "bf16"),                  # one pixel past a tile
    (4, 3, 70, 12, [-1.5, 0, 0.5, 2.25], 0, 0.5, "f32"),  # fractional shifts
    (4, 3, 70, 12, [-1.5, 0, 0.5, 2.25], 1.25, 0.75, "f16"),
    (9, 3, 200, 40, None, 0, 1, "f32"),
    (16, 2, 64, 8, list(range(-7, 9)), 0, 1, "f32"),      # largest K
    (3, 1, 1, 1, [0, 1, 2], 0, 1, "f32"),                 # one pixel, one level
    (7, 2, 257, 33, None, 3, 2, "bf16"),                  # level step 2
]


@pytest.mark.parametrize("K,H,W,D,b,dmin,dstep,st", SMALL)
@pytest.mark.parametrize("mode", ["soft", "hard"])
def test_small_cases_teacher_forced(K, H, W, D, b, dmin, dstep, st, mode):
    case = random_case(K, H, W, D, baselines=b, d_min=dmin, d_step=dstep, storage=st, mode=mode,
                       seed=K * 1000 + W)
    _say(f"small K={K} H={H} W={W} D={D} b={b} d=({dmin},{dstep}) {st} {mode}")
    teacher_forced(case, 3)


def _sobel_beyond_binary16(views):
    """Whether some 3x3 Sobel response of R+G+B (replicated border) is not
    exact in binary16 (|G| > 2048 and odd)."""
    L = np.pad(views.astype(np.int64).sum(-1), ((0, 0), (1, 1), (1, 1)), mode="edge")
    gx = (L[:, :-2, 2:] - L[:, :-2, :-2]) + 2 * (L[:, 1:-1, 2:] - L[:, 1:-1, :-2]) + (L[:, 2:, 2:] - L[:, 2:, :-2])
    gy = (L[:, 2:, :-2] - L[:, :-2, :-2]) + 2 * (L[:, 2:, 1:-1] - L[:, :-2, 1:-1]) + (L[:, 2:, 2:] - L[:, :-2, 2:])
    g = np.concatenate([gx.ravel(), gy.ravel()])
    return bool(np.any((np.abs(g) > 2048) & (g % 2 != 0)))


@pytest.mark.parametrize("K,b,dstep", [(5, None, 1), (4, [-1.5, 0, 0.5, 2.25], 0.5)])
def test_fp32_descriptors_beyond_binary16(K, b, dstep):
    """Binary views (0 or 255 per channel): Sobel responses up to 3060, many
    of them not exact in binary16, so FP32 descriptors take the int16 records."""
    case = random_case(K, 4, 150, 20, baselines=b, d_step=dstep, storage="f32", seed=31 + K)
    case.views = np.where(case.views >= 128, 255, 0).astype(np.uint8)
    assert _sobel_beyond_binary16(case.views)
    _say(f"binary views K={K} 4x150 D=20 fp32 b={b}: int16 records")
    teacher_forced(case, 3)


def test_plain_full_size_fp32():
    fr = workload_frame("plain")
    case = Case.from_frame(fr, storage="f32")
    _say("plain 640x480 K=5 D=64 fp32 soft teacher-forced x10 (full frame)")
    teacher_forced(case, 10)


def test_precision_fp16_sampled_rows():
    fr = workload_frame("precision")
    case = Case.from_frame(fr, storage="f16")
    for band in row_bands(case) + [(472, 488)]:
        _say(f"precision 1280x960 K=5 D=128 fp16 teacher-forced x10, rows {band[0]}..{band[1]}")
        teacher_forced(case, 10, rows=band)


def test_large_bf16_sampled_rows():
    fr = workload_frame("large")
    case = Case.from_frame(fr, storage="bf16")
    for band in row_bands(case) + [(530, 542)]:
        _say(f"large 1920x1080 K=9 D=192 bf16 teacher-forced x12, rows {band[0]}..{band[1]}")
        teacher_forced(case, 12, rows=band)


def test_large_fp32_sampled_rows():
    """The large frames in FP32 storage, as the plain context the server's
    BF16 streams are compared with runs them."""
    fr = workload_frame("large")
    case = Case.from_frame(fr, storage="f32")
    for band in row_bands(case)[:2]:
        _say(f"large 1920x1080 K=9 D=192 fp32 teacher-forced x12, rows {band[0]}..{band[1]}")
        teacher_forced(case, 12, rows=band)


def test_resume_is_bitwise(small_frame):
    case = Case.from_frame(small_frame, storage="f32")
    _say("small_frame resume: iterate(3)+iterate(2) vs iterate(5)")
    a = DeviceRun(case)
    a.iterate(3)
    a.iterate(2)
    qa, da, La = a.state()
    a.close()
    b = DeviceRun(case)
    b.iterate(5)
    qb, db, Lb = b.state()
    b.close()
    assert np.array_equal(qa, qb) and np.array_equal(da, db) and np.array_equal(La, Lb)


def test_host_and_device_inputs_agree(small_frame):
    case = Case.from_frame(small_frame, storage="f16")
    _say("small_frame host vs device inputs, fp16")
    a = DeviceRun(case, device_inputs=True)
    a.iterate(4)
    ra = a.refocus()
    a.close()
    b = DeviceRun(case, device_inputs=False)
    b.iterate(4)
    rb = b.refocus()
    b.close()
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)


def test_warm_start_uses_given_weights(small_frame):
    case = Case.from_frame(small_frame, storage="f32")
    _say("small_frame warm start")
    qw = np.random.default_rng(5).uniform(0, 1, (case.K, case.H, case.W)).astype(np.float32)
    run = DeviceRun(case, q_warm=qw)
    q0, _, _ = run.state(with_d=False)
    assert np.array_equal(q0, qw)
    run.iterate(1)
    q1, d1, L1 = run.state()
    run.close()
    op = case.oracle_params()
    f = O.descriptors(op, case.views)
    pr = O.ray_prior(op, case.S_P, case.mu_T)
    ref = O.em_iteration(op, f, pr[0], case.mu_T, qw.astype(np.float64), omr=pr.omr)
    tie = near_tie(ref["E1"], ref["E2"])
    assert np.all((d1 == ref["d_idx"]) | tie)


def test_frame_objective_is_sum_of_pixels(small_frame):
    case = Case.from_frame(small_frame, storage="f32")
    _say("small_frame frame objective")
    run = DeviceRun(case)
    obj = run.iterate(3, objective=True)
    q, d, L = run.state()
    run.close()
    assert abs(obj[-1] - L.astype(np.float64).sum()) <= 1e-9 * abs(obj[-1])
    assert np.all(np.diff(obj) >= -1e-6 * np.abs(obj[1:]))


def test_median_refocus(small_frame):
    case = Case.from_frame(small_frame, storage="f32")
    _say("small_frame refocus with 3x3 median")
    run = DeviceRun(case)
    run.iterate(2)
    rgb0, d, q, hole = run.refocus(median=0)
    rgb3, _, _, _ = run.refocus(median=3)
    run.close()
    op = case.oracle_params()
    want = O.median3(op, rgb0.astype(np.float64))
    assert np.array_equal(rgb3.astype(np.float64), want.astype(np.float32).astype(np.float64))


def test_device_value_validation(small_frame):
    import torch
    import paper_2003_11076_amd as LF
    case = Case.from_frame(small_frame, storage="f32")
    _say("device-side S_P validation")
    sp = case.S_P.copy()
    sp[1, 5, 7] = np.nan
    dev = torch.device("cuda")
    tv = torch.from_numpy(case.views).to(dev)
    ts = torch.from_numpy(sp).to(dev)
    tm = torch.from_numpy(case.mu_T).to(dev)
    with pytest.raises(LF.LFError) as e:
        LF.lf_em_init(case.api_params(LF.LF_INPUTS_ON_DEVICE), tv, ts, tm,
                      hip_stream=torch.cuda.current_stream().cuda_stream)
    assert e.value.status == LF.LF_EINVAL


def test_deferred_value_check(small_frame):
    """LF_DEFERRED_CHECK: loads return at once; an invalid value is reported
    by the next call that waits for the stream, once, and valid frames that
    follow load and check clean."""
    import torch
    import paper_2003_11076_amd as LF
    case = Case.from_frame(small_frame, storage="f32")
    _say("deferred device-side input check")
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    tv = torch.from_numpy(case.views).to(dev)
    good = torch.from_numpy(case.S_P).to(dev)
    sp = case.S_P.copy()
    sp[2, 9, 11] = 1.5
    bad = torch.from_numpy(sp).to(dev)
    tm = torch.from_numpy(case.mu_T).to(dev)
    flags = LF.LF_INPUTS_ON_DEVICE | LF.LF_DEFERRED_CHECK
    ctx = LF.lf_em_init(case.api_params(flags), tv, good, tm, hip_stream=stream)
    try:
        LF.lf_em_check(ctx)                                  # clean start
        LF.lf_em_load(ctx, tv, bad, tm)                      # returns without waiting
        LF.lf_em_iterate(ctx, 1)
        with pytest.raises(LF.LFError) as e:
            LF.lf_em_check(ctx)
        assert e.value.status == LF.LF_EINVAL
        with pytest.raises(LF.LFError) as e:                 # the frame was unloaded
            LF.lf_em_iterate(ctx, 1)
        assert e.value.status == LF.LF_ESTATE
        LF.lf_em_load(ctx, tv, good, tm)
        LF.lf_em_iterate(ctx, 2)
        LF.lf_em_check(ctx)                                  # reported once, then clean
        q = np.zeros((case.K, case.H, case.W), np.float32)
        LF.lf_em_state(ctx, q)
        assert np.all((q >= 0) & (q <= 1))
    finally:
        LF.lf_em_destroy(ctx)


def test_state_calls_out_of_order(small_frame):
    import paper_2003_11076_amd as LF
    case = Case.from_frame(small_frame, storage="f32")
    _say("ESTATE paths")
    run = DeviceRun(case)
    rgb = np.zeros((case.H, case.W, 3), np.float32)
    with pytest.raises(LF.LFError) as e:
        LF.lf_refocus(run.ctx, rgb)
    assert e.value.status == LF.LF_ESTATE
    with pytest.raises(LF.LFError) as e:
        LF.lf_em_state(run.ctx, d_idx=np.zeros((case.H, case.W), np.int32))
    assert e.value.status == LF.LF_ESTATE
    run.close()


def test_free_running_agreement(small_frame):
    case = Case.from_frame(small_frame, storage="f32")
    _say("small_frame free-running agreement")
    run = DeviceRun(case)
    run.iterate(case.n_iters)
    rgb, d, q, hole = run.refocus()
    run.close()
    r = O.reconstruct(case.oracle_params(), case.views, case.S_P, case.mu_T, case.n_iters)
    agree = (d == r["d_idx"]).mean()
    print(f"free-running d agreement {agree:.6f}, q max-abs {np.abs(q - r['q']).max():.3g}")
    assert agree >= 0.999


SWEEP_CASES = [
    # K, H, W, D, baselines, d_min, d_step, storage, mode
    (5, 24, 300, 32, None, 0, 1, "f32", "soft"),
    (5, 24, 300, 32, None, 0, 1, "f16", "hard"),
    (9, 8, 400, 64, None, 0, 1, "bf16", "soft"),
    (4, 6, 150, 20, [-1.5, 0, 0.5, 2.25], -1.0, 0.5, "f32", "soft"),
    (3, 6, 130, 40, [0, 1, 3], 0, 1, "f16", "soft"),
]


@pytest.mark.parametrize("K,H,W,D,b,dmin,dstep,st,mode", SWEEP_CASES)
def test_fast_sweep_matches_exhaustive_bitwise(K, H, W, D, b, dmin, dstep, st, mode):
    """The one-pass sweep with exact re-evaluation returns exactly what the
    exhaustive two-pass sweep returns (same levels, weights and objective bits)."""
    import paper_2003_11076_amd as LF
    case = random_case(K, H, W, D, baselines=b, d_min=dmin, d_step=dstep, storage=st, mode=mode, seed=7 * K + W)
    _say(f"fast vs exhaustive sweep K={K} {H}x{W} D={D} {st} {mode}")
    out = []
    for flags in (0, LF.LF_EXHAUSTIVE_SWEEP):
        run = DeviceRun(case, extra_flags=flags)
        objs = [run.iterate(1, objective=True)[0] for _ in range(4)]
        out.append(run.state() + (np.array(objs),))
        run.close()
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)


def test_fast_sweep_matches_exhaustive_small(small_frame):
    import paper_2003_11076_amd as LF
    case = Case.from_frame(small_frame, storage="f32")
    _say("small_frame fast vs exhaustive sweep, 5 iterations")
    out = []
    for flags in (0, LF.LF_EXHAUSTIVE_SWEEP):
        run = DeviceRun(case, extra_flags=flags)
        obj = run.iterate(5, objective=True)
        out.append(run.state() + (obj,))
        run.close()
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)


def _fast_vs_exhaustive(case, n_iters, extra=0):
    import paper_2003_11076_amd as LF
    out = []
    for flags in (extra, extra | LF.LF_EXHAUSTIVE_SWEEP):
        run = DeviceRun(case, extra_flags=flags)
        obj = run.iterate(n_iters, objective=True)
        out.append(run.state() + (obj,))
        run.close()
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("workload", ["plain", "precision", "large"])
def test_pruned_sweep_matches_exhaustive_on_scenes(workload):
    """Structured scenes at full size, where most pixels' seed energies bound
    the levels that can still win and the workgroups sweep those pixels in
    narrow windows: every iteration's levels, weights and objective are the
    exhaustive sweep's, bit for bit."""
    fr = workload_frame(workload)
    case = Case.from_frame(fr)
    _say(f"{workload} {case.W}x{case.H} K={case.K} D={case.D} {case.storage}: pruned fast vs exhaustive, "
         f"{case.n_iters} iterations")
    _fast_vs_exhaustive(case, case.n_iters)


@pytest.mark.parametrize("label,mu_shift,sigma,gamma,mode", [
    ("prior below the level range", -9.0, 2.0, 0.05, "soft"),
    ("prior above the level range", 30.0, 2.0, 0.05, "soft"),
    ("prior far outside the level range", -1.0e5, 2.0, 0.05, "soft"),
    ("narrow prior", 0.0, 0.35, 0.05, "soft"),
    ("prior wider than the level range", 0.0, 40.0, 0.05, "soft"),
    ("small gamma", 0.0, 2.0, 1e-6, "hard"),
    ("large gamma", 0.0, 2.0, 0.9, "soft"),
])
def test_pruned_sweep_edges_match_exhaustive(small_frame, label, mu_shift, sigma, gamma, mode):
    """Windows clipped at either end of the level range, radii from one level
    to wider than the range, and gamma from tiny to close to 1."""
    case = Case.from_frame(small_frame, storage="f32", mode=mode, sigma=np.float32(sigma),
                           gamma=np.float32(gamma))
    case.mu_T = (case.mu_T + np.float32(mu_shift)).astype(np.float32)
    _say(f"small_frame pruned fast vs exhaustive: {label} (mu {mu_shift:+}, sigma {sigma}, gamma {gamma}, {mode})")
    _fast_vs_exhaustive(case, 5)


@pytest.mark.parametrize("variant", ["dynamic-only", "window"])
def test_pruned_sweep_variants_match_exhaustive_on_scene(variant):
    import paper_2003_11076_amd as LF
    fr = workload_frame("plain")
    case = Case.from_frame(fr)
    flag = LF.LF_DYNAMIC_ONLY if variant == "dynamic-only" else LF.LF_PRIOR_WINDOW
    _say(f"plain {variant}: pruned fast vs exhaustive, 10 iterations")
    _fast_vs_exhaustive(case, 10, extra=flag)


def test_precision_fp16_error_against_unquantised_oracle():
    """Reported, not a parity bound: FP16 storage end to end (10 free-running
    iterations) against the FP64 oracle on unrounded inputs, rows 472..488."""
    fr = workload_frame("precision")
    case = Case.from_frame(fr, storage="f16")
    _say("precision fp16 end to end vs the unquantised FP64 oracle, rows 472..488")
    run = DeviceRun(case)
    run.iterate(10)
    rgb, d, q, hole = run.refocus()
    run.close()
    ref = O.reconstruct(Case.from_frame(fr, storage="f32").oracle_params(),
                        case.views, case.S_P, case.mu_T, 10, rows=(472, 488))
    y = slice(472, 488)
    agree = float((d[y] == ref["d_idx"][y]).mean())
    qerr = np.abs(q[:, y].astype(np.float64) - ref["q"][:, y])
    rerr = np.abs(rgb[y].astype(np.float64) - ref["rgb"][y])
    print(f"[report] d agreement {agree:.5f}  q max {qerr.max():.3g} p99.9 {np.percentile(qerr, 99.9):.3g}  "
          f"rgb max {rerr.max():.3g} mean {rerr.mean():.3g}", flush=True)
    assert agree > 0.98
