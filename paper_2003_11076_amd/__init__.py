"""MI355X (gfx950) EM static-background reconstruction for a linear camera array.

Thin ctypes binding of the C ABI in ``include/lf_em.h`` (``liblfem.so``, built
in-tree by ``python -m paper_2003_11076_amd.build``).  The functions keep the C
names and only marshal arguments: every step of the method runs in the HIP
kernels of the library.  Array arguments may be numpy arrays (host memory),
torch tensors (their device or host memory, by ``data_ptr``), raw integer
addresses, or None where the C function accepts NULL.  A status other than
LF_OK raises :class:`LFError` carrying the code and ``lf_last_error()``.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblfem.so")

LF_OK, LF_EINVAL, LF_ENOMEM, LF_EDEVICE, LF_EAGAIN, LF_ESTATE = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "LF_OK", 1: "LF_EINVAL", 2: "LF_ENOMEM", 3: "LF_EDEVICE", 4: "LF_EAGAIN", 5: "LF_ESTATE"}
LF_MAX_VIEWS = 16
LF_F32, LF_F16, LF_BF16 = 0, 1, 2
LF_SOFT, LF_HARD, LF_ENUM_SOFT, LF_ENUM_HARD = 0, 1, 2, 3
LF_ENUM_MAX_VIEWS = 12
MODES = {"soft": LF_SOFT, "hard": LF_HARD, "enum_soft": LF_ENUM_SOFT, "enum_hard": LF_ENUM_HARD}
LF_INPUTS_ON_DEVICE, LF_OUTPUTS_ON_DEVICE, LF_EXHAUSTIVE_SWEEP = 0x1, 0x2, 0x4
LF_PRIOR_WINDOW, LF_DYNAMIC_ONLY, LF_DEFERRED_CHECK = 0x8, 0x10, 0x20
STORAGE = {"f32": LF_F32, "f16": LF_F16, "bf16": LF_BF16}


class LFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lf_params(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("ref", ctypes.c_int32),
        ("baselines", ctypes.c_float * LF_MAX_VIEWS),
        ("d_min", ctypes.c_float), ("d_step", ctypes.c_float), ("D", ctypes.c_int32),
        ("beta", ctypes.c_float), ("lambda_", ctypes.c_float), ("gamma", ctypes.c_float),
        ("sigma", ctypes.c_float), ("tau_init", ctypes.c_float),
        ("storage", ctypes.c_int32), ("mode", ctypes.c_int32), ("flags", ctypes.c_uint32),
    ]


def make_params(K, H, W, ref, baselines, d_min, d_step, D, beta, lam=float("nan"), gamma=0.05, sigma=2.0,
                tau_init=0.7, storage="f32", mode="soft", flags=0) -> lf_params:
    p = lf_params()
    p.K, p.H, p.W, p.ref = int(K), int(H), int(W), int(ref)
    for k, b in enumerate(baselines):
        p.baselines[k] = float(b)
    p.d_min, p.d_step, p.D = float(d_min), float(d_step), int(D)
    p.beta, p.lambda_, p.gamma, p.sigma, p.tau_init = float(beta), float(lam), float(gamma), float(sigma), float(tau_init)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.flags = int(flags)
    return p


_lib = None


def lib():
    """The loaded liblfem.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2003_11076_amd.build` "
                              "(the HIP library is required; there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, P = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(lf_params)
        L.lf_em_init.argtypes = [ctypes.POINTER(vp), P, vp, vp, vp, vp, vp]
        L.lf_em_load.argtypes = [vp, vp, vp, vp, vp]
        L.lf_em_iterate.argtypes = [vp, i32, vp]
        L.lf_refocus.argtypes = [vp, vp, vp, vp, vp, i32]
        L.lf_em_state.argtypes = [vp, vp, vp, vp]
        L.lf_segmentation_maps.argtypes = [vp, vp]
        L.lf_em_check.argtypes = [vp]
        L.lf_em_intermediates.argtypes = [vp, vp, vp]
        L.lf_em_sweep_count.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint64)]
        L.lf_em_frame_noalloc.argtypes = [P, vp, vp, vp, vp, i32, vp, vp, vp, vp, i32, vp, vp, vp]
        L.lf_em_destroy.argtypes = [vp]
        L.lf_em_destroy.restype = None
        L.lf_last_error.restype = ctypes.c_char_p
        for f in ("lf_em_init", "lf_em_load", "lf_em_iterate", "lf_refocus", "lf_em_state", "lf_em_intermediates",
                  "lf_segmentation_maps", "lf_em_check", "lf_em_frame_noalloc", "lf_em_sweep_count"):
            getattr(L, f).restype = i32
        _bind_server(L)
        _bind_prior(L)
        _lib = L
    return _lib


class lf_server_stats_t(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
        ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64), ("mean_batch_frames", ctypes.c_double),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double), ("frames_per_s", ctypes.c_double),
        ("hbm_in_use", ctypes.c_int64), ("hbm_peak", ctypes.c_int64), ("max_batch_frames", ctypes.c_int64),
    ]


lf_done_fn = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p)


class lf_support_params(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int32), ("radius", ctypes.c_int32), ("texture_min", ctypes.c_int32),
        ("ratio_num", ctypes.c_int32), ("ratio_den", ctypes.c_int32), ("incon_radius", ctypes.c_int32),
        ("incon_levels", ctypes.c_int32), ("incon_min", ctypes.c_int32), ("static_min", ctypes.c_int32),
    ]


def make_support_params(step=5, radius=2, texture_min=2000, ratio_num=85, ratio_den=100, incon_radius=10,
                        incon_levels=2, incon_min=3, static_min=20) -> lf_support_params:
    sp = lf_support_params()
    sp.step, sp.radius, sp.texture_min, sp.ratio_num, sp.ratio_den = step, radius, texture_min, ratio_num, ratio_den
    sp.incon_radius, sp.incon_levels, sp.incon_min, sp.static_min = incon_radius, incon_levels, incon_min, static_min
    return sp


def _bind_prior(L):
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.lf_triangulate.argtypes = [vp, i32, vp, i32, i32p]
    L.lf_triangulate.restype = i32
    L.lf_build_prior.argtypes = [ctypes.POINTER(lf_params), ctypes.POINTER(lf_support_params), vp, vp, vp, vp, i32,
                                 i32p, vp, i32, i32p, vp]
    L.lf_build_prior.restype = i32


def lf_triangulate(xy):
    """Delaunay triangles int32 [T][3] of int32 points [n][2] (host only)."""
    xy = np.ascontiguousarray(xy, np.int32).reshape(-1, 2)
    n_t = ctypes.c_int32(0)
    _check(lib().lf_triangulate(addr(xy), len(xy), None, 0, ctypes.byref(n_t)))
    tris = np.zeros((max(n_t.value, 1), 3), np.int32)
    _check(lib().lf_triangulate(addr(xy), len(xy), addr(tris), n_t.value, ctypes.byref(n_t)))
    return tris[:n_t.value]


def lf_build_prior(p, sp, views, S_P, mu_T, max_points=0, max_tris=0, hip_stream=None):
    """Builds mu_T (written into mu_T); returns (points [n][4], tris [T][3]),
    each cut to max_points / max_tris rows (0: none returned)."""
    n_p, n_t = ctypes.c_int32(0), ctypes.c_int32(0)
    pts = np.zeros((max(max_points, 1), 4), np.int32)
    tris = np.zeros((max(max_tris, 1), 3), np.int32)
    _check(lib().lf_build_prior(ctypes.byref(p), ctypes.byref(sp), addr(views), addr(S_P), addr(mu_T),
                                addr(pts) if max_points else None, max_points, ctypes.byref(n_p),
                                addr(tris) if max_tris else None, max_tris, ctypes.byref(n_t), hip_stream))
    return pts[:min(n_p.value, max_points)], tris[:min(n_t.value, max_tris)], n_p.value, n_t.value


def _bind_server(L):
    vp, i32, P = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(lf_params)
    L.lf_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, i32, i32, ctypes.c_size_t]
    L.lf_submit_frame.argtypes = [vp, i32, P, vp, vp, vp, vp, vp, vp, lf_done_fn, vp, ctypes.POINTER(ctypes.c_int64)]
    L.lf_server_drain.argtypes = [vp]
    L.lf_server_hold.argtypes = [vp, i32]
    L.lf_server_stats.argtypes = [vp, ctypes.POINTER(lf_server_stats_t)]
    L.lf_server_reset_stats.argtypes = [vp]
    L.lf_server_destroy.argtypes = [vp]
    L.lf_server_destroy.restype = None
    for f in ("lf_server_create", "lf_submit_frame", "lf_server_drain", "lf_server_stats", "lf_server_reset_stats",
              "lf_server_hold"):
        getattr(L, f).restype = i32


def last_error() -> str:
    return lib().lf_last_error().decode()


lf_last_error = last_error


def _check(status):
    if status != LF_OK:
        raise LFError(status, last_error())
    return status


def addr(x):
    """Address of an array argument (numpy, torch, int) or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):          # torch tensor
        if not x.is_contiguous():
            raise ValueError("tensor arguments must be contiguous")
        return x.data_ptr()
    if hasattr(x, "ctypes"):            # numpy array
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array arguments must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"cannot pass {type(x)!r} as an array")


def lf_em_init(p: lf_params, views, S_P, mu_T, q_warm=None, hip_stream=None) -> int:
    """Returns the context handle (an int)."""
    out = ctypes.c_void_p()
    _check(lib().lf_em_init(ctypes.byref(out), ctypes.byref(p), addr(views), addr(S_P), addr(mu_T), addr(q_warm),
                            hip_stream))
    return out.value


def lf_em_load(ctx, views, S_P, mu_T, q_warm=None):
    return _check(lib().lf_em_load(ctx, addr(views), addr(S_P), addr(mu_T), addr(q_warm)))


def lf_em_iterate(ctx, n_iters, objective=None):
    return _check(lib().lf_em_iterate(ctx, int(n_iters), addr(objective)))


def lf_refocus(ctx, rgb, d_idx=None, q=None, hole=None, median=0):
    return _check(lib().lf_refocus(ctx, addr(rgb), addr(d_idx), addr(q), addr(hole), int(median)))


def lf_em_state(ctx, q=None, d_idx=None, L_pix=None):
    return _check(lib().lf_em_state(ctx, addr(q), addr(d_idx), addr(L_pix)))


def lf_em_sweep_count(ctx, n_iters) -> int:
    """Runs n_iters iterations; returns the sweeps' level steps summed over waves."""
    v = ctypes.c_uint64(0)
    _check(lib().lf_em_sweep_count(ctx, int(n_iters), ctypes.byref(v)))
    return v.value


def lf_em_check(ctx):
    return _check(lib().lf_em_check(ctx))


def lf_segmentation_maps(ctx, labels):
    return _check(lib().lf_segmentation_maps(ctx, addr(labels)))


def lf_em_intermediates(ctx, feat=None, rho=None):
    return _check(lib().lf_em_intermediates(ctx, addr(feat), addr(rho)))


LF_NOALLOC_SCRATCH_BYTES = 64 << 20


def lf_em_frame_noalloc(p: lf_params, views, S_P, mu_T, q_warm, n_iters, rgb, d_idx, q, hole=None, median=0,
                        objective=None, invalid=None, hip_stream=None):
    """One whole frame with no allocation; every array is device memory."""
    return _check(lib().lf_em_frame_noalloc(ctypes.byref(p), addr(views), addr(S_P), addr(mu_T), addr(q_warm),
                                            int(n_iters), addr(rgb), addr(d_idx), addr(q), addr(hole), int(median),
                                            addr(objective), addr(invalid), hip_stream))


def lf_em_destroy(ctx):
    if ctx:
        lib().lf_em_destroy(ctx)


def lf_server_create(hbm_budget_bytes, max_streams, n_iters, staging_bytes=0) -> int:
    out = ctypes.c_void_p()
    _check(lib().lf_server_create(ctypes.byref(out), int(hbm_budget_bytes), int(max_streams), int(n_iters),
                                  int(staging_bytes)))
    return out.value


def lf_submit_frame(srv, stream_id, p: lf_params, views, S_P, mu_T, rgb_out, d_out=None, q_out=None, done=None,
                    user=None) -> int:
    """`done` must be an lf_done_fn the caller keeps alive until it has run."""
    fid = ctypes.c_int64(-1)
    _check(lib().lf_submit_frame(srv, int(stream_id), ctypes.byref(p), addr(views), addr(S_P), addr(mu_T),
                                 addr(rgb_out), addr(d_out), addr(q_out), done if done is not None else lf_done_fn(),
                                 user, ctypes.byref(fid)))
    return fid.value


def lf_server_hold(srv, hold):
    return _check(lib().lf_server_hold(srv, int(bool(hold))))


def lf_server_drain(srv):
    return _check(lib().lf_server_drain(srv))


def lf_server_stats(srv) -> lf_server_stats_t:
    st = lf_server_stats_t()
    _check(lib().lf_server_stats(srv, ctypes.byref(st)))
    return st


def lf_server_reset_stats(srv):
    return _check(lib().lf_server_reset_stats(srv))


def lf_server_destroy(srv):
    if srv:
        lib().lf_server_destroy(srv)
