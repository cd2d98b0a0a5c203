"""Parity of the enumeration E-step (ENUM_SOFT / ENUM_HARD: all 2^K labelings
with the coupled variance, Sec. III-C last sentence and Sec. III-D) against
the FP64 oracle, through the C ABI.  Tolerances are those of tests/lfcase.py;
enumerated hard labels are exempt only where the two largest labeling log
weights are within 1e-3."""
import sys

import numpy as np
import pytest

import lf_scenes as S
from lfcase import Case, DeviceRun, random_case, teacher_forced, workload_frame

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["enum_soft", "enum_hard"])
def test_small_scene_enumeration_teacher_forced(mode):
    case = Case.from_frame(S.make_frame(S.workload_spec("small")), storage="f32", mode=mode)
    _say(f"small_frame 160x120 K=5 D=32 fp32 {mode} teacher-forced x3")
    teacher_forced(case, 3)


SMALL = [
    # K, H, W, D, baselines, d_min, d_step, storage
    (2, 5, 37, 9, [0, 1], 0, 1, "f32"),
    (3, 4, 300, 16, [-1, 0, 2], -2, 1, "f16"),
    (5, 3, 129, 24, None, 0, 1, "bf16"),
    (4, 3, 70, 12, [-1.5, 0, 0.5, 2.25], 0, 0.5, "f32"),
    (7, 2, 257, 33, None, 3, 2, "bf16"),
    (9, 2, 140, 20, None, 0, 1, "f32"),
    (12, 1, 64, 8, list(range(-5, 7)), 0, 1, "f16"),     # largest K of the enumeration
]


@pytest.mark.parametrize("K,H,W,D,b,dmin,dstep,st", SMALL)
@pytest.mark.parametrize("mode", ["enum_soft", "enum_hard"])
def test_small_enumeration_teacher_forced(K, H, W, D, b, dmin, dstep, st, mode):
    case = random_case(K, H, W, D, baselines=b, d_min=dmin, d_step=dstep, storage=st, mode=mode,
                       beta=400.0, seed=K * 1000 + W + 7)
    _say(f"enum small K={K} H={H} W={W} D={D} b={b} d=({dmin},{dstep}) {st} {mode}")
    teacher_forced(case, 2)


def test_large_enumeration_sampled_rows():
    case = Case.from_frame(workload_frame("large"), storage="bf16", mode="enum_soft")
    _say("large 1920x1080 K=9 D=192 bf16 enum_soft teacher-forced x2, rows 536..539")
    teacher_forced(case, 2, rows=(536, 539))


def test_enumeration_fast_sweep_matches_exhaustive():
    """The enumeration modes change only the E-step: the fast and the
    exhaustive sweep still give the same bits."""
    import paper_2003_11076_amd as LF
    case = random_case(5, 6, 200, 32, storage="f16", mode="enum_soft", seed=77)
    _say("enum_soft fast vs exhaustive sweep K=5 6x200 D=32 f16")
    outs = []
    for flags in (0, LF.LF_EXHAUSTIVE_SWEEP):
        run = DeviceRun(case, extra_flags=flags)
        run.iterate(3)
        outs.append(run.state())
        run.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
