"""The paper's further outputs through the C ABI: the refocused image after
every EM iteration (Sec. III-E: it is computed at each iteration) and the
per-view segmentation maps in each view's own grid (Sec. III-D), against the
FP64 oracle on the GPU's own levels and weights."""
import sys

import numpy as np
import pytest

import lf_scenes as S
import oracle as O
from lfcase import Case, DeviceRun, random_case, TOL_RGB

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _labels(run):
    c = run.case
    lab = np.full((c.K, c.H, c.W), 255, np.uint8)
    run.LF.lf_segmentation_maps(run.ctx, lab)
    return lab


def _half_pixel_exempt(case, d_idx):
    """[K][H][W] view pixels a ray reaches from within 1e-6 of a half pixel."""
    ex = np.zeros((case.K, case.H, case.W), bool)
    xs = np.arange(case.W, dtype=np.float64)
    for k in range(case.K):
        u = xs[None, :] - case.baselines[k] * (case.d_min + d_idx.astype(np.float64) * case.d_step)
        near = np.abs(u - np.floor(u) - 0.5) < 1e-6
        for y, x in zip(*np.nonzero(near)):
            for v in (int(np.floor(u[y, x])), int(np.floor(u[y, x])) + 1):
                if 0 <= v < case.W:
                    ex[k, y, v] = True
    return ex


CASES = [
    ("small_frame", None),
    ("small", dict(K=4, H=5, W=150, D=20, baselines=[-1.5, 0, 0.5, 2.25], d_min=-1.0, d_step=0.5, storage="f32")),
    ("small", dict(K=7, H=3, W=300, D=40, storage="bf16")),
    ("small", dict(K=3, H=4, W=90, D=16, storage="f16", baselines=[0, 1, 3])),
]


@pytest.mark.parametrize("name,kw", CASES)
def test_per_iteration_refocus_and_segmentation(name, kw):
    if kw is None:
        case = Case.from_frame(S.make_frame(S.workload_spec("small")), storage="f32")
    else:
        kw = dict(kw)
        case = random_case(kw.pop("K"), kw.pop("H"), kw.pop("W"), kw.pop("D"), seed=31, **kw)
    _say(f"per-iteration refocus and segmentation maps: {name} K={case.K} {case.H}x{case.W} D={case.D}")
    op = case.oracle_params()
    run = DeviceRun(case)
    try:
        for t in range(3):
            run.iterate(1)
            rgb, d, q, hole = run.refocus()
            rgb_o, hole_o = O.refocus(op, case.views, d, q.astype(np.float64))
            assert np.array_equal(hole, hole_o), t
            near_half = (np.abs(q.astype(np.float64) - 0.5) < 1e-4).any(axis=0)
            rd = np.abs(rgb.astype(np.float64) - rgb_o).max(axis=-1)[~near_half]
            assert rd.size == 0 or rd.max() <= TOL_RGB, (t, rd.max())
            lab = _labels(run)
            lab_o = O.segmentation_maps(op, d, q.astype(np.float64))
            # same levels and weights on both sides: labels are exact, except
            # where a ray reaches a view within 1e-6 of a half pixel
            ex = _half_pixel_exempt(case, d)
            bad = (lab != lab_o) & ~ex
            assert not bad.any(), (t, np.argwhere(bad)[:5].tolist())
            assert set(np.unique(lab)) <= {0, 1, 2}
    finally:
        run.close()


def test_refocus_between_iterations_leaves_the_state_alone():
    case = random_case(5, 6, 200, 32, storage="f16", seed=32)
    _say("iterate(1) + refocus + iterate(1) == iterate(2), bitwise")
    a = DeviceRun(case)
    a.iterate(1)
    a.refocus()
    _labels(a)
    a.iterate(1)
    sa = a.state()
    a.close()
    b = DeviceRun(case)
    b.iterate(2)
    sb = b.state()
    b.close()
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
