"""FP64 CPU oracle of the EM static-background light-field reconstruction.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never calls it and
shares no code with it; the oracle is plain C (``lf_oracle.c``) in double
precision, wrapped here with ctypes, plus these thin numpy conveniences.

Every function follows the paper (Kaveti, Katt and Singh, 2020):
  descriptors  -> Sec. III-C, pixel likelihood (3x3 Sobel responses)
  ray_prior    -> Sec. III-B (S_P prior of each view) and Sec. III-F (0.7 threshold)
  em_iteration -> Sec. III-B (EM schedule, M-step first), Sec. III-C (E(d), Eq. 6),
                  Sec. III-D (segmentation posterior, Eq. 7)
  refocus      -> Eq. 2 (static rays only) and Sec. IV-B (no static ray: keep the pixel)
  median3      -> Sec. III-E (median filter against the refocus' specular noise)
  segmentation_maps -> Sec. III-D (updated segmentation, shown per view in its own grid)
  support_points, raster_prior -> Sec. III-C (disparity prior: support points, dynamic filtering,
                  transfer from the other views, triangulation and interpolation)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lf_oracle.c")
_LIB = os.path.join(_HERE, "liblforacle.so")
MAX_VIEWS = 16
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
# soft / hard: per-view posterior of the factorised model; enum_*: the paper's
# enumeration of all labelings with the coupled variance (marginals / arg max)
MODES = {"soft": 0, "hard": 1, "enum_soft": 2, "enum_hard": 3}


class Params(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("ref", ctypes.c_int32),
        ("baselines", ctypes.c_double * MAX_VIEWS),
        ("d_min", ctypes.c_double), ("d_step", ctypes.c_double), ("D", ctypes.c_int32),
        ("beta", ctypes.c_double), ("lam", ctypes.c_double), ("gamma", ctypes.c_double),
        ("sigma", ctypes.c_double), ("tau", ctypes.c_double),
        ("storage", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("window", ctypes.c_double), ("dyn_only", ctypes.c_int32),
    ]


def make_params(K, H, W, ref, baselines, d_min, d_step, D, beta, lam=float("nan"), gamma=0.05,
                sigma=2.0, tau=0.7, storage="f32", mode="soft", window=0.0, dyn_only=False) -> Params:
    p = Params()
    p.K, p.H, p.W, p.ref = K, H, W, ref
    for k, b in enumerate(baselines):
        p.baselines[k] = float(b)
    p.d_min, p.d_step, p.D = float(d_min), float(d_step), int(D)
    p.beta, p.lam, p.gamma, p.sigma, p.tau = float(beta), float(lam), float(gamma), float(sigma), float(tau)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.window, p.dyn_only = float(window), int(bool(dyn_only))
    return p


class SupportParams(ctypes.Structure):
    """Support-point matching and filtering parameters (prior construction)."""
    _fields_ = [
        ("step", ctypes.c_int32), ("radius", ctypes.c_int32), ("texture_min", ctypes.c_int32),
        ("ratio_num", ctypes.c_int32), ("ratio_den", ctypes.c_int32),
        ("incon_radius", ctypes.c_int32), ("incon_levels", ctypes.c_int32), ("incon_min", ctypes.c_int32),
        ("static_min", ctypes.c_int32),
    ]


def make_support_params(step=5, radius=2, texture_min=2000, ratio_num=85, ratio_den=100, incon_radius=10,
                        incon_levels=2, incon_min=3, static_min=20) -> SupportParams:
    sp = SupportParams()
    sp.step, sp.radius, sp.texture_min = step, radius, texture_min
    sp.ratio_num, sp.ratio_den = ratio_num, ratio_den
    sp.incon_radius, sp.incon_levels, sp.incon_min = incon_radius, incon_levels, incon_min
    sp.static_min = static_min
    return sp


def build(force: bool = False) -> str:
    """Compile lf_oracle.c with gcc (no HIP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.POINTER(Params)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i32 = ctypes.c_int32
        L.lfo_round_storage.argtypes = [ctypes.c_double, i32]
        L.lfo_round_storage.restype = ctypes.c_double
        L.lfo_derive_lambda.argtypes = [P]
        L.lfo_derive_lambda.restype = ctypes.c_double
        L.lfo_descriptors.argtypes = [P, u8, dp, i32, i32]
        L.lfo_ray_prior.argtypes = [P, fp, fp, dp, dp, dp, i32, i32]
        L.lfo_em_iteration.argtypes = [P, ctypes.c_double, dp, dp, dp, fp, dp, dp, i32p, dp, dp, dp, i32, i32]
        L.lfo_refocus.argtypes = [P, u8, i32p, dp, dp, dp, u8, i32, i32]
        L.lfo_reconstruct.argtypes = [P, u8, fp, fp, dp, i32, i32, i32, dp, dp, dp, dp, dp, i32p, dp, dp, dp, u8]
        L.lfo_reconstruct.restype = i32
        L.lfo_threads.restype = i32
        L.lfo_median3.argtypes = [P, dp, dp, i32, i32]
        L.lfo_segmentation_maps.argtypes = [P, i32p, dp, u8, i32, i32]
        L.lfo_support_points.argtypes = [P, ctypes.POINTER(SupportParams), u8, fp, i32p, i32]
        L.lfo_support_points.restype = i32
        L.lfo_raster_prior.argtypes = [P, i32p, i32, i32p, i32, fp]
        L.lfo_prior_corners.argtypes = [P, i32p, i32]
        L.lfo_prior_corners.restype = i32
        _lib = L
    return _lib


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ct))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _rows(p, rows):
    return (0, p.H) if rows is None else (int(rows[0]), int(rows[1]))


def round_storage(v, storage) -> float:
    return lib().lfo_round_storage(float(v), STORAGE[storage] if isinstance(storage, str) else int(storage))


def derive_lambda(p: Params) -> float:
    return lib().lfo_derive_lambda(ctypes.byref(p))


def lam_of(p: Params) -> float:
    return derive_lambda(p) if math.isnan(p.lam) else p.lam


def descriptors(p: Params, views, rows=None) -> np.ndarray:
    """[K][H][W][2] float64 descriptors (rows outside `rows` are zero)."""
    v = _c(views, np.uint8)
    f = np.zeros((p.K, p.H, p.W, 2), np.float64)
    y0, y1 = _rows(p, rows)
    lib().lfo_descriptors(ctypes.byref(p), _ptr(v, ctypes.c_uint8), _ptr(f, ctypes.c_double), y0, y1)
    return f


class RayPrior(tuple):
    """(rho, q0) with the dynamic prior omr = 1 - rho as an attribute."""
    omr: np.ndarray


def ray_prior(p: Params, S_P, mu_T, rows=None):
    """(rho, q0): [K][H][W] float64 each; `.omr` holds 1 - rho interpolated
    from 1 - S_P (accurate where rho is close to 1)."""
    sp, mu = _c(S_P, np.float32), _c(mu_T, np.float32)
    rho = np.zeros((p.K, p.H, p.W))
    omr = np.ones((p.K, p.H, p.W))
    q0 = np.zeros((p.K, p.H, p.W))
    y0, y1 = _rows(p, rows)
    lib().lfo_ray_prior(ctypes.byref(p), _ptr(sp, ctypes.c_float), _ptr(mu, ctypes.c_float),
                        _ptr(rho, ctypes.c_double), _ptr(omr, ctypes.c_double), _ptr(q0, ctypes.c_double), y0, y1)
    out = RayPrior((rho, q0))
    out.omr = omr
    return out


def em_iteration(p: Params, f, rho, mu_T, q_in, lam=None, rows=None, omr=None) -> dict:
    """One EM iteration (M-step, then E-step) from weights q_in.  omr is the
    dynamic prior 1 - rho (taken as 1 - rho when None).

    Returns q [K][H][W], d_idx [H][W], L [H][W] (per-pixel objective after the
    E-step), E1/E2 [H][W] (smallest and second smallest M-step energies)."""
    lam = lam_of(p) if lam is None else float(lam)
    f, rho, mu, q_in = _c(f, np.float64), _c(rho, np.float64), _c(mu_T, np.float32), _c(q_in, np.float64)
    omr = None if omr is None else _c(omr, np.float64)
    out = {
        "q": np.zeros((p.K, p.H, p.W)), "d_idx": np.zeros((p.H, p.W), np.int32),
        "L": np.zeros((p.H, p.W)), "E1": np.zeros((p.H, p.W)), "E2": np.zeros((p.H, p.W)),
    }
    y0, y1 = _rows(p, rows)
    D = ctypes.c_double
    lib().lfo_em_iteration(ctypes.byref(p), lam, _ptr(f, D), _ptr(rho, D), _ptr(omr, D), _ptr(mu, ctypes.c_float),
                           _ptr(q_in, D), _ptr(out["q"], D), _ptr(out["d_idx"], ctypes.c_int32),
                           _ptr(out["L"], D), _ptr(out["E1"], D), _ptr(out["E2"], D), y0, y1)
    return out


def refocus(p: Params, views, d_idx, q, rows=None, rho=None):
    """(rgb [H][W][3] in [0,1], hole [H][W] uint8).  rho (the ray prior) is
    needed only with dyn_only, to find the pixels with a static reference ray."""
    v, d, q = _c(views, np.uint8), _c(d_idx, np.int32), _c(q, np.float64)
    rho = None if rho is None else _c(rho, np.float64)
    rgb = np.zeros((p.H, p.W, 3))
    hole = np.zeros((p.H, p.W), np.uint8)
    y0, y1 = _rows(p, rows)
    lib().lfo_refocus(ctypes.byref(p), _ptr(v, ctypes.c_uint8), _ptr(d, ctypes.c_int32),
                      _ptr(q, ctypes.c_double), _ptr(rho, ctypes.c_double), _ptr(rgb, ctypes.c_double),
                      _ptr(hole, ctypes.c_uint8), y0, y1)
    return rgb, hole


def segmentation_maps(p: Params, d_idx, q, rows=None):
    """Per-view labels uint8 [K][H][W] in each view's own grid: 1 static,
    0 dynamic, 2 no reference ray lands there (nearest surface wins)."""
    d, q = _c(d_idx, np.int32), _c(q, np.float64)
    labels = np.full((p.K, p.H, p.W), 255, np.uint8)
    y0, y1 = _rows(p, rows)
    lib().lfo_segmentation_maps(ctypes.byref(p), _ptr(d, ctypes.c_int32), _ptr(q, ctypes.c_double),
                                _ptr(labels, ctypes.c_uint8), y0, y1)
    return labels


def support_points(p: Params, sp: SupportParams, views, S_P) -> np.ndarray:
    """Support points int32 [n][4] = (u, y, level, view), sorted by (y, u)."""
    v, s = _c(views, np.uint8), _c(S_P, np.float32)
    nx = max(0, (p.W - sp.step // 2 + sp.step - 1) // sp.step)
    ny = max(0, (p.H - sp.step // 2 + sp.step - 1) // sp.step)
    cap = nx * ny * p.K + 1
    out = np.zeros((cap, 4), np.int32)
    n = lib().lfo_support_points(ctypes.byref(p), ctypes.byref(sp), _ptr(v, ctypes.c_uint8), _ptr(s, ctypes.c_float),
                                 _ptr(out, ctypes.c_int32), cap)
    if n < 0:
        raise ValueError("bad support parameters")
    return out[:n].copy()


def prior_corners(p: Params, points) -> np.ndarray:
    """points plus the four image corners (view -1) at the level of the
    nearest support point, corners already present skipped."""
    pts = np.zeros((len(points) + 4, 4), np.int32)
    pts[:len(points)] = points
    n = lib().lfo_prior_corners(ctypes.byref(p), _ptr(pts, ctypes.c_int32), len(points))
    return pts[:n].copy()


def raster_prior(p: Params, points, tris) -> np.ndarray:
    """mu_T float32 [H][W] from support points and a triangulation of them."""
    pts, tr = _c(points, np.int32), _c(np.asarray(tris, np.int32).reshape(-1, 3), np.int32)
    mu = np.zeros((p.H, p.W), np.float32)
    lib().lfo_raster_prior(ctypes.byref(p), _ptr(pts, ctypes.c_int32), len(pts), _ptr(tr, ctypes.c_int32), len(tr),
                           _ptr(mu, ctypes.c_float))
    return mu


def median3(p: Params, rgb, rows=None):
    """3x3 per-channel median with replicated border, [H][W][3] float64."""
    src = _c(rgb, np.float64)
    out = np.zeros((p.H, p.W, 3))
    y0, y1 = _rows(p, rows)
    lib().lfo_median3(ctypes.byref(p), _ptr(src, ctypes.c_double), _ptr(out, ctypes.c_double), y0, y1)
    return out


def reconstruct(p: Params, views, S_P, mu_T, n_iters, q_warm=None, rows=None) -> dict:
    """Whole method on rows [y0, y1): descriptors, ray prior, n_iters EM
    iterations, refocus.  Returns q, d_idx, L (last iteration, per pixel),
    L_sum (per iteration, plain sum), rgb, hole, threads."""
    v, sp, mu = _c(views, np.uint8), _c(S_P, np.float32), _c(mu_T, np.float32)
    K, H, W = p.K, p.H, p.W
    qw = None if q_warm is None else _c(q_warm, np.float64)
    f = np.zeros((K, H, W, 2))
    rho = np.zeros((K, H, W))
    omr = np.ones((K, H, W))
    qa = np.zeros((K, H, W))
    qb = np.zeros((K, H, W))
    d = np.zeros((H, W), np.int32)
    L = np.zeros((H, W))
    Ls = np.zeros(max(1, n_iters))
    rgb = np.zeros((H, W, 3))
    hole = np.zeros((H, W), np.uint8)
    y0, y1 = _rows(p, rows)
    D = ctypes.c_double
    th = lib().lfo_reconstruct(ctypes.byref(p), _ptr(v, ctypes.c_uint8), _ptr(sp, ctypes.c_float),
                               _ptr(mu, ctypes.c_float), _ptr(qw, D), int(n_iters), y0, y1,
                               _ptr(f, D), _ptr(rho, D), _ptr(omr, D), _ptr(qa, D), _ptr(qb, D),
                               _ptr(d, ctypes.c_int32), _ptr(L, D), _ptr(Ls, D), _ptr(rgb, D),
                               _ptr(hole, ctypes.c_uint8))
    return {"q": qa, "d_idx": d, "L": L, "L_sum": Ls[:n_iters], "rgb": rgb, "hole": hole,
            "threads": th, "f": f, "rho": rho}


def threads() -> int:
    return lib().lfo_threads()
