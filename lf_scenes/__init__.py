"""Seeded synthetic light-field frames for a rectified horizontal camera array.

This module is input generation only.  It renders K rectified views of a
static background built from planes plus fronto-parallel dynamic objects, the
per-view semantic segmentation prior S_P (probability of *static*, so
S_P = 0 means dynamic, Sec. III-B) and a dense disparity prior mu_T standing
in for the triangulation of sparse support points (Sec. III-C, "Disparity
Prior").  It contains none of the reconstruction method's arithmetic (no
descriptors, no EM, no refocus) and is the only module shared by the FP64
oracle tests and the GPU path.

Geometry.  View k samples the reference pixel (u, y) at x = u - b_k * delta,
so a view pixel (x, y) sees reference coordinate u = x + b_k * delta(u, y).
For a plane delta = a + bu*u + c*y this solves to
u = (x + b_k*(a + c*y)) / (1 - b_k*bu).  Among the surfaces whose solution
falls inside their own support, the one with the largest disparity (the
closest) is visible.  The paper's own data (720x540 indoor/outdoor sequences
with people, Sec. IV-B) is not available; these scenes stand in for it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Frame", "SceneSpec", "make_frame", "workload_spec", "WORKLOAD_NAMES", "WORKLOADS",
    "serving_stream_spec", "rng_for", "frame_arrays",
]

# Largest |G| of a 3x3 Sobel response of L = R+G+B (4 * 765), and the scale
# that maps integer responses into descriptor units.  Used only to choose beta.
_DESC_SCALE = 2.0 ** -12


def rng_for(base: int, tag: int, k: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (scene base seed, purpose tag, index)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([base, tag, k])))


# Purpose tags for rng_for.
_T_TEXTURE, _T_PLACE, _T_NOISE, _T_SP, _T_T = 1, 2, 3, 4, 5


# ---------------------------------------------------------------------------
# Textures
# ---------------------------------------------------------------------------

def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _gradient_noise_grid(ny, nx, period, rng):
    """2-D gradient noise (Perlin) on the integer grid [0,ny) x [0,nx) with a
    seeded lattice of random unit gradients every `period` (integer) pixels.
    Evaluated cell by cell with broadcasting.  Values roughly in [-0.7, 0.7]."""
    P = int(period)
    cj, ci = -(-ny // P), -(-nx // P)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(cj + 1, ci + 1))
    gx, gy = np.cos(ang), np.sin(ang)
    gx, gy = gx.astype(np.float32), gy.astype(np.float32)
    t = (np.arange(P) / P).astype(np.float32)
    fu = t[None, None, None, :]
    fy = t[None, None, :, None]

    def corner(di, dj):
        g_x = gx[dj:dj + cj, di:di + ci][:, :, None, None]
        g_y = gy[dj:dj + cj, di:di + ci][:, :, None, None]
        return g_x * (fu - di) + g_y * (fy - dj)

    n00, n10, n01, n11 = corner(0, 0), corner(1, 0), corner(0, 1), corner(1, 1)
    su, sy = _fade(fu), _fade(fy)
    nx0 = n00 + su * (n10 - n00)
    nx1 = n01 + su * (n11 - n01)
    n = nx0 + sy * (nx1 - nx0)                      # [cj][ci][P][P]
    n = n.transpose(0, 2, 1, 3).reshape(cj * P, ci * P)
    return n[:ny, :nx]


def _perlin_texture(H, u_lo, u_hi, rng, period=32, octaves=3):
    """RGB texture image over integer u in [u_lo, u_hi] and rows 0..H-1:
    `octaves` octaves of gradient noise, base period `period` px, per channel."""
    nx = u_hi - u_lo + 1
    out = np.empty((H, nx, 3), np.float64)
    for ch in range(3):
        acc = np.zeros((H, nx))
        amp, per = 1.0, period
        for _ in range(octaves):
            acc += amp * _gradient_noise_grid(H, nx, per, rng)
            amp *= 0.5
            per //= 2
        out[:, :, ch] = np.clip(0.5 + 0.6 * acc, 0.0, 1.0)
    return out


def _iid_texture(H, u_lo, u_hi, rng):
    """iid U[0,1]^3 per texel over integer u in [u_lo, u_hi]."""
    return rng.uniform(0.0, 1.0, size=(H, u_hi - u_lo + 1, 3))


@dataclass
class _Tex:
    img: np.ndarray  # [H][n_u][3] in [0,1]
    u_lo: int

    def sample(self, u, y):
        """Linear interpolation along u (exact at integer u); rows are integer."""
        n = self.img.shape[1]
        t = u - self.u_lo
        i0 = np.floor(t).astype(np.int64)
        fr = (t - i0)[..., None]
        i0c = np.clip(i0, 0, n - 1)
        i1c = np.clip(i0 + 1, 0, n - 1)
        yy = y.astype(np.int64)
        return (1.0 - fr) * self.img[yy, i0c] + fr * self.img[yy, i1c]


# ---------------------------------------------------------------------------
# Surfaces
# ---------------------------------------------------------------------------

@dataclass
class _Surface:
    static: bool
    a: float            # disparity = a + bu*u + c*y (reference coordinates)
    bu: float = 0.0
    c: float = 0.0
    kind: str = "cell"  # "cell" (Voronoi cell of the background), "rect", "ellipse"
    geom: tuple = ()
    tex: _Tex | None = None

    def solve_u(self, x, y, b):
        return (x + b * (self.a + self.c * y)) / (1.0 - b * self.bu)

    def disparity(self, u, y):
        return self.a + self.bu * u + self.c * y


def _support(s: _Surface, u, y, cell_of):
    if s.kind == "cell":
        return cell_of(u, y) == s.geom[0]
    if s.kind == "rect":
        u0, y0, w, h = s.geom
        return (u >= u0) & (u < u0 + w) & (y >= y0) & (y < y0 + h)
    if s.kind == "ellipse":
        cx, cy, rx, ry = s.geom
        return ((u - cx) / rx) ** 2 + ((y - cy) / ry) ** 2 <= 1.0
    raise ValueError(s.kind)


# ---------------------------------------------------------------------------
# Public types
# ---------------------------------------------------------------------------

@dataclass
class SceneSpec:
    """Everything that defines one synthetic frame and its method parameters."""
    name: str
    K: int
    H: int
    W: int
    baselines: tuple
    ref: int
    D: int
    n_iters: int
    d_min: float = 0.0
    d_step: float = 1.0
    sigma: float = 2.0
    gamma: float = 0.05
    tau: float = 0.7
    storage: str = "f32"          # "f32", "f16", "bf16"
    texture: str = "iid"          # "iid" or "perlin"
    n_planes: int = 1
    slanted: bool = False
    bg_disp: tuple = (6, 6)       # background disparity range
    dyn_kind: str = "rect"        # "rect", "ellipse", "mixed"
    n_dyn: int = 1
    dyn_disp: tuple = (20, 20)
    dyn_cover: tuple = (0.15, 0.15)  # accepted union coverage range
    noise_sigma: float = 0.0      # photometric noise, in [0,1] units
    sp_model: str = "gauss"       # "gauss": clip(M + N(0, 0.1^2)); "blurflip": blur 2px + 10% flips
    n_T: int = 30
    seed: int = 1000
    beta: float | None = None     # None -> chosen from the noise-free texture
    dyn_shift: float = 0.0        # dynamic objects' horizontal offset (serving streams)


@dataclass
class Frame:
    spec: SceneSpec
    views: np.ndarray        # uint8 [K][H][W][3]
    S_P: np.ndarray          # float32 [K][H][W], probability of static
    mu_T: np.ndarray         # float32 [H][W], dense prior disparity
    baselines: np.ndarray    # float32 [K]
    beta: float
    # ground truth (sanity checks only)
    disp_bg: np.ndarray      # float64 [H][W] true static-background disparity (reference view)
    mask: np.ndarray         # uint8 [K][H][W] true static mask of each view
    bg_rgb: np.ndarray       # float64 [H][W][3] noise-free background colour (reference view)
    extras: dict = field(default_factory=dict)

    @property
    def K(self):
        return self.spec.K

    @property
    def H(self):
        return self.spec.H

    @property
    def W(self):
        return self.spec.W


# ---------------------------------------------------------------------------
# Scene construction
# ---------------------------------------------------------------------------

def _voronoi(sites):
    sx = np.array([s[0] for s in sites])[:, None]
    sy = np.array([s[1] for s in sites])[:, None]

    def cell_of(u, y):
        shp = np.shape(u)
        uu = np.ravel(u)[None, :]
        yy = np.ravel(y)[None, :]
        d2 = (uu - sx) ** 2 + (yy - sy) ** 2
        return np.argmin(d2, axis=0).reshape(shp)
    return cell_of


def _build_surfaces(spec: SceneSpec):
    rng_p = rng_for(spec.seed, _T_PLACE)
    H, W = spec.H, spec.W
    sites = [(rng_p.uniform(0, W), rng_p.uniform(0, H)) for _ in range(spec.n_planes)]
    cell_of = _voronoi(sites)
    bg = []
    lo, hi = spec.bg_disp
    for i in range(spec.n_planes):
        if spec.slanted:
            # disparity at the frame corners uniform in [lo, hi]; three are drawn
            # and redrawn until the fourth (planar) corner is in range as well
            while True:
                d00, d10, d01 = rng_p.uniform(lo, hi, size=3)
                if lo <= d10 + d01 - d00 <= hi:
                    break
            bu = (d10 - d00) / (W - 1)
            c = (d01 - d00) / (H - 1)
            a = d00
        else:
            a = float(rng_p.integers(lo, hi + 1)) if spec.n_planes > 1 else float(lo)
            bu = c = 0.0
        bmax = max(abs(b) for b in spec.baselines)
        assert abs(bmax * bu) < 0.5
        bg.append(_Surface(True, a, bu, c, "cell", (i,)))

    # dynamic objects: resample placements until the union coverage (reference
    # view) is inside the requested range
    dyn = []
    cov_lo, cov_hi = spec.dyn_cover
    target = 0.5 * (cov_lo + cov_hi)
    # coverage is measured on a 1/4-subsampled grid for large frames
    st = 4 if H * W > 1_000_000 else 1
    ys, xs = np.mgrid[0:H:st, 0:W:st].astype(np.float64)
    for attempt in range(2000):
        dyn = []
        for o in range(spec.n_dyn):
            kind = spec.dyn_kind
            if kind == "mixed":
                kind = "rect" if o % 2 == 0 else "ellipse"
            dlo, dhi = spec.dyn_disp
            dd = float(rng_p.integers(int(dlo), int(dhi) + 1)) if spec.texture == "iid" \
                else float(rng_p.uniform(dlo, dhi))
            area = target * H * W / spec.n_dyn * rng_p.uniform(0.8, 1.25)
            if spec.n_dyn == 1 and kind == "rect":
                # exact-size rectangle (48x60 at 160x120 covers 15.0%)
                w = int(round(math.sqrt(area * 0.8)))
                h = int(round(area / w))
                u0 = int(rng_p.integers(0, W - w + 1))
                y0 = int(rng_p.integers(0, H - h + 1))
                geom = (u0 + spec.dyn_shift, y0, w, h)
            elif kind == "rect":
                w = max(4, int(round(math.sqrt(area * rng_p.uniform(0.5, 1.5)))))
                h = max(4, int(round(area / w)))
                w, h = min(w, W - 1), min(h, H - 1)
                u0 = int(rng_p.integers(0, W - w + 1))
                y0 = int(rng_p.integers(0, H - h + 1))
                geom = (u0 + spec.dyn_shift, y0, w, h)
            else:
                ar = rng_p.uniform(0.5, 1.5)
                rx = math.sqrt(area * ar / math.pi)
                ry = area / (math.pi * rx)
                rx, ry = min(rx, W / 2), min(ry, H / 2)
                cx = rng_p.uniform(rx * 0.5, W - rx * 0.5)
                cy = rng_p.uniform(ry * 0.5, H - ry * 0.5)
                geom = (cx + spec.dyn_shift, cy, rx, ry)
            dyn.append(_Surface(False, dd, 0.0, 0.0, kind, geom))
        cov = np.zeros(xs.shape, bool)
        for s in dyn:
            cov |= _support(s, xs, ys, cell_of)
        frac = cov.mean()
        if cov_lo - 1e-9 <= frac <= cov_hi + 1e-9:
            break
    else:
        raise RuntimeError(f"could not place dynamic objects for {spec.name}")
    return bg, dyn, cell_of


def _attach_textures(spec: SceneSpec, surfaces):
    bmax = max(abs(b) for b in spec.baselines)
    dmax = spec.d_min + spec.d_step * (spec.D - 1)
    margin = int(math.ceil(bmax * max(dmax, max(abs(s.a) + abs(s.bu) * spec.W + abs(s.c) * spec.H
                                                     for s in surfaces)))) + 4
    u_lo, u_hi = -margin, spec.W - 1 + margin
    for i, s in enumerate(surfaces):
        rng_t = rng_for(spec.seed, _T_TEXTURE, i)
        if spec.texture == "iid":
            img = _iid_texture(spec.H, u_lo, u_hi, rng_t)
        else:
            img = _perlin_texture(spec.H, u_lo, u_hi, rng_t)
        s.tex = _Tex(img, u_lo)


def _render(spec: SceneSpec, bg, dyn, cell_of):
    K, H, W = spec.K, spec.H, spec.W
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    surfaces = bg + dyn
    views = np.empty((K, H, W, 3), np.uint8)
    mask = np.empty((K, H, W), np.uint8)
    for k in range(K):
        b = float(spec.baselines[k])
        best_disp = np.full((H, W), -np.inf)
        best_idx = np.full((H, W), -1, np.int64)
        best_u = np.zeros((H, W))
        far_disp = np.full((H, W), np.inf)
        far_idx = np.zeros((H, W), np.int64)
        far_u = np.zeros((H, W))
        for si, s in enumerate(surfaces):
            u = s.solve_u(xs, ys, b)
            dsp = s.disparity(u, ys)
            ok = _support(s, u, ys, cell_of)
            upd = ok & (dsp > best_disp)
            best_disp = np.where(upd, dsp, best_disp)
            best_idx = np.where(upd, si, best_idx)
            best_u = np.where(upd, u, best_u)
            if s.static:
                fu = dsp < far_disp
                far_disp = np.where(fu, dsp, far_disp)
                far_idx = np.where(fu, si, far_idx)
                far_u = np.where(fu, u, far_u)
        # disocclusion gaps: fall back to the farthest background plane
        gap = best_idx < 0
        best_idx = np.where(gap, far_idx, best_idx)
        best_u = np.where(gap, far_u, best_u)
        col = np.zeros((H, W, 3))
        for si, s in enumerate(surfaces):
            sel = best_idx == si
            if sel.any():
                col[sel] = s.tex.sample(best_u[sel], ys[sel])
        if spec.noise_sigma > 0:
            col = col + rng_for(spec.seed, _T_NOISE, k).normal(0.0, spec.noise_sigma, size=col.shape)
        views[k] = np.round(255.0 * np.clip(col, 0.0, 1.0)).astype(np.uint8)
        mask[k] = np.array([1 if s.static else 0 for s in surfaces], np.uint8)[best_idx]
    # reference-view background truth: the static plane whose cell holds (x, y)
    cell = cell_of(xs, ys)
    disp_bg = np.zeros((H, W))
    bg_rgb = np.zeros((H, W, 3))
    for i, s in enumerate(bg):
        sel = cell == i
        disp_bg[sel] = s.disparity(xs[sel], ys[sel])
        bg_rgb[sel] = s.tex.sample(xs[sel], ys[sel])
    return views, mask, disp_bg, bg_rgb


def _segmentation_prior(spec: SceneSpec, mask):
    """Per-view P(static) from the true mask (stands in for a CNN, Sec. III-F)."""
    rng = rng_for(spec.seed, _T_SP)
    m = mask.astype(np.float64)
    if spec.sp_model == "gauss":
        sp = np.clip(m + rng.normal(0.0, 0.1, size=m.shape), 0.0, 1.0)
    elif spec.sp_model == "blurflip":
        from scipy.ndimage import gaussian_filter
        sp = np.stack([gaussian_filter(m[k], 2.0, mode="nearest") for k in range(m.shape[0])])
        flip = rng.uniform(size=sp.shape) < 0.10
        sp = np.where(flip, 1.0 - sp, sp)
        sp = np.clip(sp, 0.0, 1.0)
    else:
        raise ValueError(spec.sp_model)
    return sp.astype(np.float32)


def _prior_map(spec: SceneSpec, disp_bg):
    """Dense mu_T: piecewise-linear interpolation over a Delaunay triangulation
    of n_T sparse true background disparities, nearest sample outside the hull."""
    from scipy.interpolate import LinearNDInterpolator, NearestNDInterpolator
    H, W = spec.H, spec.W
    rng = rng_for(spec.seed, _T_T)
    idx = rng.choice(H * W, size=spec.n_T, replace=False)
    py, px = np.divmod(idx, W)
    pts = np.stack([px, py], axis=1).astype(np.float64)
    vals = disp_bg[py, px]
    ys, xs = np.mgrid[0:H, 0:W]
    q = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float64)
    if np.ptp(vals) == 0.0:
        mu = np.full(H * W, vals[0])
    else:
        lin = LinearNDInterpolator(pts, vals)(q)
        near = NearestNDInterpolator(pts, vals)(q)
        mu = np.where(np.isnan(lin), near, lin)
    return mu.reshape(H, W).astype(np.float32)


def _beta_from_texture(spec: SceneSpec, bg_rgb):
    """beta = 40*K / ((K-1) * F * v_tex), v_tex = per-dimension variance of the
    noise-free reference texture's Sobel responses (scipy's), in descriptor units."""
    if spec.texture == "iid":
        # analytic: L = R+G+B of iid uniform bytes; Sobel gain 12 on var(L)
        v_tex = 12.0 * 3.0 * ((256.0 ** 2 - 1.0) / 12.0) * _DESC_SCALE ** 2
    else:
        from scipy.ndimage import sobel
        L = np.round(255.0 * bg_rgb).sum(axis=2)
        gx = sobel(L, axis=1, mode="nearest") * _DESC_SCALE
        gy = sobel(L, axis=0, mode="nearest") * _DESC_SCALE
        v_tex = 0.5 * (gx[1:-1, 1:-1].var() + gy[1:-1, 1:-1].var())
    F = 2
    return 40.0 * spec.K / ((spec.K - 1) * F * v_tex)


def make_frame(spec: SceneSpec) -> Frame:
    bg, dyn, cell_of = _build_surfaces(spec)
    _attach_textures(spec, bg + dyn)
    views, mask, disp_bg, bg_rgb = _render(spec, bg, dyn, cell_of)
    S_P = _segmentation_prior(spec, mask)
    mu_T = _prior_map(spec, disp_bg)
    beta = spec.beta if spec.beta is not None else _beta_from_texture(spec, bg_rgb)
    return Frame(spec, views, S_P, mu_T, np.asarray(spec.baselines, np.float32), float(beta),
                 disp_bg, mask, bg_rgb,
                 extras={"dyn_disp": [s.a for s in dyn], "bg_planes": [(s.a, s.bu, s.c) for s in bg]})


# ---------------------------------------------------------------------------
# The workloads: four single-frame scenes and the serving stream mix
# ---------------------------------------------------------------------------

WORKLOAD_NAMES = {
    "small": "plain-em-fp64-160x120-k5-d32-i5",
    "plain": "plain-em-fp32-640x480-k5-d64-i10",
    "precision": "precision-fp16-1280x960-k5-d128-i10",
    "serving": "serving-mix-fp16-i8",
    "large": "large-bf16-1920x1080-k9-d192-i12",
}
WORKLOADS = ("small", "plain", "precision", "large")   # single-frame scenes
# seed bases of the scenes (every draw of a scene is seeded from its base)
_SEED_BASE = {"small": 1000, "plain": 2000, "precision": 3000, "large": 5000}


def _sym(K):
    return tuple(float(k - (K - 1) // 2) for k in range(K))


def workload_spec(name: str, **over) -> SceneSpec:
    """SceneSpec of a single-frame workload: "small", "plain", "precision" or
    "large" (the serving mix is serving_stream_spec)."""
    if name not in WORKLOADS:
        raise ValueError(f"{name!r} is not a single-frame workload ({', '.join(WORKLOADS)})")
    base = _SEED_BASE[name]
    if name == "small":
        s = SceneSpec(WORKLOAD_NAMES["small"], K=5, H=120, W=160, baselines=_sym(5), ref=2, D=32,
                      n_iters=5, texture="iid", n_planes=1, bg_disp=(6, 6), dyn_kind="rect",
                      n_dyn=1, dyn_disp=(20, 20), dyn_cover=(0.15, 0.15), noise_sigma=0.0,
                      sp_model="gauss", n_T=30, seed=base, beta=2133.0)
    elif name == "plain":
        s = SceneSpec(WORKLOAD_NAMES["plain"], K=5, H=480, W=640, baselines=_sym(5), ref=2, D=64,
                      n_iters=10, texture="perlin", n_planes=4, slanted=True, bg_disp=(2, 20),
                      dyn_kind="ellipse", n_dyn=3, dyn_disp=(25, 50), dyn_cover=(0.20, 0.40),
                      noise_sigma=2.0 / 255.0, sp_model="blurflip", n_T=200, seed=base)
    elif name == "precision":
        s = SceneSpec(WORKLOAD_NAMES["precision"], K=5, H=960, W=1280, baselines=_sym(5), ref=2, D=128,
                      n_iters=10, storage="f16", texture="iid", n_planes=6, bg_disp=(2, 40),
                      dyn_kind="mixed", n_dyn=5, dyn_disp=(50, 120), dyn_cover=(0.34, 0.36),
                      noise_sigma=0.0, sp_model="gauss", n_T=1920, seed=base, beta=2133.0)
    elif name == "large":
        s = SceneSpec(WORKLOAD_NAMES["large"], K=9, H=1080, W=1920, baselines=_sym(9), ref=4, D=192,
                      n_iters=12, storage="bf16", texture="perlin", n_planes=6, slanted=True,
                      bg_disp=(4, 60), dyn_kind="mixed", n_dyn=5, dyn_disp=(70, 180),
                      dyn_cover=(0.49, 0.51), noise_sigma=2.0 / 255.0, sp_model="blurflip",
                      n_T=1350, seed=base)
    for k, v in over.items():
        setattr(s, k, v)
    return s


# Serving mix: per-stream fixed shapes so that warm start applies.
_SERVE_SIZES = [(240, 320)] * 5 + [(480, 640)] * 8 + [(960, 1280)] * 3


def serving_stream_spec(stream: int, frame: int, scale: float = 1.0) -> SceneSpec:
    """Frame `frame` of serving stream `stream` (0..15): sizes 320x240/640x480/
    1280x960 for 5/8/3 streams, K cycling 3/5/7 and D cycling 32/64/128 at
    offset phases, FP16 storage, 8 EM iterations, objects moving 2 px/frame.
    `scale` < 1 shrinks the frame (tests)."""
    H, W = _SERVE_SIZES[stream % len(_SERVE_SIZES)]
    H, W = max(16, int(H * scale)), max(32, int(W * scale))
    K = (3, 5, 7)[stream % 3]
    D = (32, 64, 128)[(stream // 3 + stream) % 3]
    return SceneSpec(f"serve-s{stream}-f{frame}", K=K, H=H, W=W, baselines=_sym(K), ref=(K - 1) // 2,
                     D=D, n_iters=8, storage="f16", texture="perlin", n_planes=3, slanted=True,
                     bg_disp=(2, max(3, int(0.3 * D))), dyn_kind="ellipse", n_dyn=2,
                     dyn_disp=(int(0.4 * D), int(0.8 * D)), dyn_cover=(0.10, 0.45),
                     noise_sigma=2.0 / 255.0, sp_model="blurflip", n_T=max(20, H * W // 1536),
                     seed=40000 + 100 * stream, dyn_shift=2.0 * frame)


def frame_arrays(spec: SceneSpec):
    """(views, S_P, mu_T, beta) of make_frame(spec): the arrays a caller of
    the library needs, small enough to hand back from a worker process."""
    fr = make_frame(spec)
    return fr.views, fr.S_P, fr.mu_T, float(fr.beta)
