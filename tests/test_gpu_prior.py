"""Construction of the disparity prior on the GPU (lf_build_prior, Sec. III-C)
against the oracle: the support points (integer work: exact), the corners,
a valid Delaunay triangulation of them (several are correct where points are
cocircular, so the GPU's own is checked by definition), and mu_T against the
oracle's raster of that triangulation."""
import sys

import numpy as np
import pytest

import lf_scenes as S
import oracle as O
from lfcase import f32
from test_triangulation import _check_delaunay, _hull

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _run(spec, fr, check_all_circles):
    import torch
    import paper_2003_11076_amd as LF
    K, H, W = spec.K, spec.H, spec.W
    p = LF.make_params(K, H, W, spec.ref, spec.baselines, spec.d_min, spec.d_step, spec.D, fr.beta,
                       tau_init=spec.tau)
    sp = LF.make_support_params()
    mu = np.zeros((H, W), np.float32)
    cap_p, cap_t = ((W // 5 + 1) * (H // 5 + 1) * K + 8), 4 * (W // 5 + 1) * (H // 5 + 1) * K + 16
    pts, tris, n_p, n_t = LF.lf_build_prior(p, sp, fr.views, fr.S_P, mu, cap_p, cap_t,
                                            hip_stream=torch.cuda.current_stream().cuda_stream)
    assert len(pts) == n_p and len(tris) == n_t
    op = O.make_params(K, H, W, spec.ref, [f32(b) for b in spec.baselines], f32(spec.d_min), f32(spec.d_step),
                       spec.D, f32(fr.beta), tau=f32(spec.tau))
    ref = O.prior_corners(op, O.support_points(op, O.make_support_params(), fr.views, fr.S_P))
    assert np.array_equal(pts, ref)
    if check_all_circles:
        _check_delaunay(pts[:, :2], tris)
    else:
        _, h, area2 = _hull(pts[:, :2].tolist())
        assert n_t == 2 * len(pts) - h - 2
        a, b, c = pts[tris[:, 0], :2].astype(np.int64), pts[tris[:, 1], :2].astype(np.int64), pts[tris[:, 2], :2].astype(np.int64)
        o = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
        assert np.all(o > 0) and o.sum() == area2
    mu_o = O.raster_prior(op, pts, tris)
    assert np.array_equal(mu, mu_o)
    return pts, mu


def test_prior_small():
    fr = S.make_frame(S.workload_spec("small"))
    _say("build prior small_frame 160x120 K=5 D=32")
    pts, mu = _run(fr.spec, fr, True)
    assert np.abs(mu - fr.disp_bg).max() == 0.0          # one plane: recovered exactly


def test_prior_plain():
    fr = S.make_frame(S.workload_spec("plain"))
    _say("build prior plain 640x480 K=5 D=64")
    pts, mu = _run(fr.spec, fr, False)
    err = np.abs(mu - fr.disp_bg)
    assert np.percentile(err, 50) < 1.0                  # sanity against the scene's truth


def test_prior_small_asymmetric():
    spec = S.workload_spec("small", H=60, W=100, baselines=(0.0, 1.0, 2.0, 3.0, 4.0), ref=0, dyn_kind="ellipse",
                         dyn_cover=(0.05, 0.4))
    fr = S.make_frame(spec)
    _say("build prior 100x60 K=5 reference at the end of the array")
    _run(spec, fr, True)


def _points_only(K, H, W, b, D, ref, views, S_P, **spkw):
    """The GPU's points for a synthetic scene against the oracle's (support
    points with the corners), exact."""
    import torch
    import paper_2003_11076_amd as LF
    p = LF.make_params(K, H, W, ref, b, 0.0, 1.0, D, 100.0)
    sp = LF.make_support_params(**spkw)
    mu = np.zeros((H, W), np.float32)
    cap = (W // 5 + 1) * (H // 5 + 1) * K + 8
    pts, tris, n_p, n_t = LF.lf_build_prior(p, sp, views, S_P, mu, cap, 4 * cap + 16,
                                            hip_stream=torch.cuda.current_stream().cuda_stream)
    op = O.make_params(K, H, W, ref, [f32(v) for v in b], f32(0.0), f32(1.0), D, f32(100.0))
    want = O.prior_corners(op, O.support_points(op, O.make_support_params(**spkw), views, S_P))
    assert np.array_equal(pts, want)
    return pts


def test_prior_points_moved_onto_one_pixel():
    """Every non-reference view's grid points land on the same reference
    pixels (plane at a multiple of the grid step): one point per pixel, from
    the lowest view, as the oracle."""
    from test_oracle_pins import _plane_views
    rng = np.random.default_rng(74)
    K, H, W, D, d0 = 5, 40, 100, 16, 5
    b = [-2.0, -1.0, 0.0, 1.0, 2.0]
    views = _plane_views(K, H, W, b, d0, rng)
    views[2, 10:30, 40:70] = rng.integers(0, 256, size=(20, 30, 3))
    S_P = np.ones((K, H, W), np.float32)
    S_P[2, 10:30, 40:70] = 0.0
    _say("prior: moved points colliding on reference pixels, K=5 100x40")
    pts = _points_only(K, H, W, b, D, 2, views, S_P)
    assert (pts[:, 3] == 0).sum() > 20


@pytest.mark.parametrize("incon_levels,incon_min", [(2, 8), (2, 12), (1, 8), (3, 12), (2, 0)])
def test_prior_consistency_bounds(incon_levels, incon_min):
    """Two planes exactly incon_levels apart and minimum counts around the
    number of neighbours: the consistency filter's bounds, as the oracle."""
    rng = np.random.default_rng(73)
    K, H, W, D = 3, 40, 90, 16
    b = [-1.0, 0.0, 1.0]
    pad = 12
    tex = rng.integers(0, 256, size=(H, W + 2 * pad, 3))
    views = np.zeros((K, H, W, 3), np.uint8)
    for k in range(K):
        for x in range(W):
            d = 4 if x < W // 2 else 6
            views[k, :, x] = tex[:, pad + x + int(b[k]) * d]
    ones = np.ones((K, H, W), np.float32)
    _say(f"prior: consistency incon_levels={incon_levels} incon_min={incon_min}")
    _points_only(K, H, W, b, D, 1, views, ones, incon_levels=incon_levels, incon_min=incon_min)


def test_prior_wide_consistency_radius():
    """A consistency radius of several grid rows (the device scans each row
    in range by binary search)."""
    fr = S.make_frame(S.workload_spec("small"))
    spec = fr.spec
    _say("prior: small_frame with incon_radius=23, incon_min=30")
    _points_only(spec.K, spec.H, spec.W, list(spec.baselines), spec.D, spec.ref, fr.views, fr.S_P,
                 incon_radius=23, incon_min=30)


def test_prior_device_buffers_equal_host_buffers():
    """Views and S_P in device memory and mu_T written there: the points,
    the triangles and mu_T of the host-buffer call, bit for bit."""
    import torch
    import paper_2003_11076_amd as LF
    fr = S.make_frame(S.workload_spec("small"))
    spec = fr.spec
    K, H, W = spec.K, spec.H, spec.W
    cap = (W // 5 + 1) * (H // 5 + 1) * K + 8
    st = torch.cuda.current_stream().cuda_stream
    _say("build prior small_frame: device buffers vs host buffers")
    p = LF.make_params(K, H, W, spec.ref, spec.baselines, spec.d_min, spec.d_step, spec.D, fr.beta, tau_init=spec.tau)
    mu_h = np.zeros((H, W), np.float32)
    pts_h, tris_h, _, _ = LF.lf_build_prior(p, LF.make_support_params(), fr.views, fr.S_P, mu_h, cap, 4 * cap,
                                            hip_stream=st)
    dev = torch.device("cuda:0")
    views, sp_d = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (fr.views, fr.S_P))
    mu_d = torch.full((H, W), -1.0, device=dev)
    torch.cuda.synchronize()
    pd = LF.make_params(K, H, W, spec.ref, spec.baselines, spec.d_min, spec.d_step, spec.D, fr.beta,
                        tau_init=spec.tau, flags=LF.LF_INPUTS_ON_DEVICE | LF.LF_OUTPUTS_ON_DEVICE)
    pts_d, tris_d, _, _ = LF.lf_build_prior(pd, LF.make_support_params(), views, sp_d, mu_d, cap, 4 * cap,
                                            hip_stream=st)
    torch.cuda.synchronize()
    assert np.array_equal(pts_h, pts_d) and np.array_equal(tris_h, tris_d)
    assert np.array_equal(mu_h, mu_d.cpu().numpy())
