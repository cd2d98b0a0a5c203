"""The C ABI library loads, exports every entry point include/*.h declares, and
rejects invalid arguments before any device work (runs without a GPU)."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

import paper_2003_11076_amd as LF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(lf_[a-z0-9_]+)\s*\(", src, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("lf_em_init", "lf_em_load", "lf_em_iterate", "lf_refocus", "lf_em_state",
                     "lf_em_destroy", "lf_last_error", "lf_server_create", "lf_submit_frame",
                     "lf_server_drain", "lf_server_destroy"):
        assert required in names, required


def test_library_exports_every_declared_symbol():
    lib = LF.lib()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _frame(K=3, H=4, W=10):
    views = np.zeros((K, H, W, 3), np.uint8)
    S_P = np.full((K, H, W), 0.5, np.float32)
    mu = np.zeros((H, W), np.float32)
    return views, S_P, mu


def _params(**over):
    kw = dict(K=3, H=4, W=10, ref=1, baselines=[-1, 0, 1], d_min=0, d_step=1, D=4, beta=100.0)
    kw.update(over)
    return LF.make_params(**kw)


@pytest.mark.parametrize("over,msg", [
    (dict(K=1, baselines=[0]), "K="),
    (dict(K=17, baselines=[0] * 16), "K="),
    (dict(ref=3), "ref="),
    (dict(baselines=[-1, 0.5, 1]), "baselines[ref]"),
    (dict(D=0), "D="),
    (dict(d_step=0.0), "d_step"),
    (dict(d_step=-1.0), "d_step"),
    (dict(beta=-1.0), "beta"),
    (dict(beta=0.0), "lambda"),
    (dict(gamma=0.0), "gamma"),
    (dict(sigma=0.0), "sigma"),
    (dict(tau_init=1.5), "tau_init"),
    (dict(storage=3), "storage"),
    (dict(mode=4), "mode"),
    (dict(mode=-1), "mode"),
    (dict(K=13, ref=6, baselines=list(range(-6, 7)), mode=2), "enumeration"),
    (dict(K=13, ref=6, baselines=list(range(-6, 7)), mode=3), "enumeration"),
    (dict(flags=0x40), "flags"),
    (dict(H=0), "H="),
    (dict(baselines=[-1, 0, float("inf")]), "baselines[2]"),
])
def test_invalid_params_rejected(over, msg):
    K = over.get("K", 3)
    H = over.get("H", 4) or 1
    views, S_P, mu = _frame(K=max(K, 1), H=H)
    with pytest.raises(LF.LFError) as e:
        LF.lf_em_init(_params(**over), views, S_P, mu)
    assert e.value.status == LF.LF_EINVAL
    assert msg in LF.last_error()


@pytest.mark.parametrize("what", ["sp_nan", "sp_high", "sp_low", "mu_inf", "qw_bad"])
def test_invalid_host_values_rejected(what):
    views, S_P, mu = _frame()
    qw = None
    if what == "sp_nan":
        S_P[1, 2, 3] = np.nan
    elif what == "sp_high":
        S_P[0, 0, 0] = 1.0001
    elif what == "sp_low":
        S_P[2, 3, 9] = -1e-7
    elif what == "mu_inf":
        mu[1, 1] = np.inf
    else:
        qw = np.full((3, 4, 10), 0.5, np.float32)
        qw[0, 0, 0] = 2.0
    with pytest.raises(LF.LFError) as e:
        LF.lf_em_init(_params(), views, S_P, mu, qw)
    assert e.value.status == LF.LF_EINVAL


def test_missing_inputs_and_null_handles():
    views, S_P, mu = _frame()
    with pytest.raises(LF.LFError) as e:
        LF.lf_em_init(_params(), views, None, mu)
    assert e.value.status == LF.LF_EINVAL
    lib = LF.lib()
    assert lib.lf_em_iterate(None, 1, None) == LF.LF_EINVAL
    assert lib.lf_refocus(None, None, None, None, None, 0) == LF.LF_EINVAL
    assert lib.lf_em_state(None, None, None, None) == LF.LF_EINVAL
    assert lib.lf_em_load(None, None, None, None, None) == LF.LF_EINVAL
    lib.lf_em_destroy(None)          # no-op
    out = ctypes.c_void_p(1234)
    assert lib.lf_em_init(ctypes.byref(out), None, None, None, None, None, None) == LF.LF_EINVAL
    assert out.value is None         # *out cleared on failure


def test_params_struct_layout_matches_header():
    # 4 ints, 16 floats, 2 floats, 1 int, 5 floats, 2 ints, 1 uint = 31 4-byte fields
    assert ctypes.sizeof(LF.lf_params) == 4 * 31
    assert LF.lf_params.baselines.offset == 16
    assert LF.lf_params.flags.offset == 4 * 30


def test_nan_lambda_is_the_derivation_flag():
    p = _params()
    assert math.isnan(p.lambda_)


def test_server_argument_checks_without_device():
    out = ctypes.c_void_p()
    lib = LF.lib()
    assert lib.lf_server_create(ctypes.byref(out), 1 << 30, 0, 8, 0) == LF.LF_EINVAL
    assert lib.lf_server_create(ctypes.byref(out), 1 << 30, 4, -1, 0) == LF.LF_EINVAL
    assert lib.lf_server_create(ctypes.byref(out), 1000, 4, 8, 0) == LF.LF_EINVAL   # below 64 KiB
    assert lib.lf_server_create(None, 1 << 30, 4, 8, 0) == LF.LF_EINVAL
    assert lib.lf_submit_frame(None, 0, None, None, None, None, None, None, None, LF.lf_done_fn(), None,
                               None) == LF.LF_EINVAL
    assert lib.lf_server_drain(None) == LF.LF_EINVAL
    lib.lf_server_destroy(None)
