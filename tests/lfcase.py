"""Test plumbing shared by the parity tests.

A `Case` holds one seeded frame and its parameters, rounded to float32
exactly as the C ABI receives them, so the oracle and the GPU library see the
same numbers.  `teacher_forced` runs the GPU library one EM iteration at a
time and, at every iteration, runs the FP64 oracle from the GPU's own state,
comparing element by element:

  * descriptors: bit-exact (integer Sobel, one rounding to the storage format);
  * rho: max-abs 1e-6;  first weights q0: exact except |rho - tau| < 1e-6;
  * d_idx: exact except near-ties, E_(2) - E_(1) <= 1e-4 * max(|E_(2)|, 1)
    with the oracle's two smallest energies of that iteration;
  * q: max-abs 1e-5 on pixels with matching d (hard mode: exact except
    |a1 - a0| < 1e-3, the decision taken in different precisions; enumerated
    hard labels: exact except where the two largest labeling log weights are
    within 1e-3);
  * per-pixel objective: |diff| <= 1e-5 * max(A, 1) on pixels with matching d,
    A = |ln prior| + sum_k (max(|a1_k|, |a0_k|) + ln 2) the magnitude of its
    addends (>= |L|; the FP32 rounding error scales with the addends, which
    cancel in the sum);
  * variants (window, dynamic-only): d also exempt where mu_T puts a level
    within 1e-4 of the window's edge or half-way between two levels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

import oracle as O

TOL_RHO = 1e-6
TOL_Q = 1e-5
TOL_L = 1e-5
TOL_RGB = 1e-6
NEAR_TIE = 1e-4


def f32(v) -> float:
    return float(np.float32(v))


@dataclass
class Case:
    K: int
    H: int
    W: int
    ref: int
    baselines: tuple
    d_min: float
    d_step: float
    D: int
    beta: float
    lam: float
    gamma: float
    sigma: float
    tau: float
    storage: str
    mode: str
    views: np.ndarray
    S_P: np.ndarray
    mu_T: np.ndarray
    n_iters: int = 1
    flags: int = 0          # LF_PRIOR_WINDOW / LF_DYNAMIC_ONLY (the variants), passed to both sides

    @classmethod
    def from_arrays(cls, spec, views, S_P, mu_T, beta, storage=None, mode="soft", **over):
        c = cls(spec.K, spec.H, spec.W, spec.ref, tuple(f32(b) for b in spec.baselines), f32(spec.d_min),
                f32(spec.d_step), spec.D, f32(beta), float("nan"), f32(spec.gamma), f32(spec.sigma), f32(spec.tau),
                storage or spec.storage, mode, views, S_P.astype(np.float32), mu_T.astype(np.float32), spec.n_iters)
        for k, v in over.items():
            setattr(c, k, v)
        return c

    @classmethod
    def from_frame(cls, fr, storage=None, mode="soft", **over):
        sp = fr.spec
        c = cls(sp.K, sp.H, sp.W, sp.ref, tuple(f32(b) for b in sp.baselines), f32(sp.d_min), f32(sp.d_step),
                sp.D, f32(fr.beta), float("nan"), f32(sp.gamma), f32(sp.sigma), f32(sp.tau),
                storage or sp.storage, mode, fr.views, fr.S_P.astype(np.float32), fr.mu_T.astype(np.float32),
                sp.n_iters)
        for k, v in over.items():
            setattr(c, k, v)
        return c

    def api_params(self, flags=0):
        import paper_2003_11076_amd as LF
        return LF.make_params(self.K, self.H, self.W, self.ref, self.baselines, self.d_min, self.d_step, self.D,
                              self.beta, self.lam, self.gamma, self.sigma, self.tau, self.storage, self.mode,
                              flags | self.flags)

    @property
    def window(self):
        # the C ABI's LF_PRIOR_WINDOW searches |d - mu| <= 3 sigma (sigma in float32)
        return 3.0 * f32(self.sigma) if self.flags & 0x8 else 0.0

    @property
    def dyn_only(self):
        return bool(self.flags & 0x10)

    def oracle_params(self, mode=None):
        return O.make_params(self.K, self.H, self.W, self.ref, self.baselines, self.d_min, self.d_step, self.D,
                             self.beta, self.lam, self.gamma, self.sigma, self.tau, self.storage, mode or self.mode,
                             window=f32(self.window), dyn_only=self.dyn_only)


def random_case(K, H, W, D, *, baselines=None, d_min=0.0, d_step=1.0, storage="f32", mode="soft", beta=2133.0,
                seed=0, mu_range=None, ref=None):
    """Small random-texture case (iid views, noisy S_P, smooth random mu_T)."""
    rng = np.random.default_rng(seed)
    if baselines is None:
        baselines = [float(k - (K - 1) // 2) for k in range(K)]
    if ref is None:
        ref = int(np.argmin(np.abs(np.asarray(baselines))))
    views = rng.integers(0, 256, size=(K, H, W, 3), dtype=np.uint8)
    S_P = np.clip(rng.integers(0, 2, size=(K, H, W)) + rng.normal(0, 0.15, size=(K, H, W)), 0, 1).astype(np.float32)
    lo, hi = mu_range or (d_min, d_min + d_step * (D - 1))
    mu = (rng.uniform(lo, hi) + rng.normal(0, 0.5, size=(H, W)).cumsum(axis=1) * 0.1).astype(np.float32)
    return Case(K, H, W, ref, tuple(f32(b) for b in baselines), f32(d_min), f32(d_step), D, f32(beta),
                float("nan"), f32(0.05), f32(2.0), f32(0.7), storage, mode, views, S_P, mu)


# ---------------------------------------------------------------------------
# Storage decoding
# ---------------------------------------------------------------------------

def decode_feat(raw: np.ndarray, storage: str, K, H, W) -> np.ndarray:
    """GPU descriptor bytes -> float64 [K][H][W][2]."""
    if storage == "f32":
        return raw.view(np.float32).reshape(K, H, W, 2).astype(np.float64)
    if storage == "f16":
        return raw.view(np.float16).reshape(K, H, W, 2).astype(np.float64)
    u = raw.view(np.uint16).reshape(K, H, W, 2).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def feat_bytes(storage, K, H, W):
    return K * H * W * (8 if storage == "f32" else 4)


# ---------------------------------------------------------------------------
# GPU runs through the C ABI (inputs as device tensors on torch's stream)
# ---------------------------------------------------------------------------

class DeviceRun:
    def __init__(self, case: Case, device_inputs=True, q_warm=None, extra_flags=0):
        import torch
        import paper_2003_11076_amd as LF
        self.LF, self.case = LF, case
        flags = (LF.LF_INPUTS_ON_DEVICE if device_inputs else 0) | extra_flags
        stream = torch.cuda.current_stream().cuda_stream
        if device_inputs:
            dev = torch.device("cuda")
            self.t_views = torch.from_numpy(np.ascontiguousarray(case.views)).to(dev)
            self.t_sp = torch.from_numpy(np.ascontiguousarray(case.S_P)).to(dev)
            self.t_mu = torch.from_numpy(np.ascontiguousarray(case.mu_T)).to(dev)
            self.t_qw = None if q_warm is None else torch.from_numpy(np.ascontiguousarray(q_warm, np.float32)).to(dev)
            args = (self.t_views, self.t_sp, self.t_mu, self.t_qw)
        else:
            qw = None if q_warm is None else np.ascontiguousarray(q_warm, np.float32)
            args = (np.ascontiguousarray(case.views), np.ascontiguousarray(case.S_P),
                    np.ascontiguousarray(case.mu_T), qw)
        self.ctx = LF.lf_em_init(case.api_params(flags), *args, hip_stream=stream)

    def close(self):
        if self.ctx:
            self.LF.lf_em_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def iterate(self, n, objective=False):
        obj = np.zeros(max(n, 1), np.float64) if objective else None
        self.LF.lf_em_iterate(self.ctx, n, obj)
        return obj

    def state(self, with_d=True):
        c = self.case
        q = np.zeros((c.K, c.H, c.W), np.float32)
        d = np.zeros((c.H, c.W), np.int32) if with_d else None
        L = np.zeros((c.H, c.W), np.float32) if with_d else None
        self.LF.lf_em_state(self.ctx, q, d, L)
        return q, d, L

    def intermediates(self):
        c = self.case
        raw = np.zeros(feat_bytes(c.storage, c.K, c.H, c.W), np.uint8)
        rho = np.zeros((c.K, c.H, c.W), np.float32)
        self.LF.lf_em_intermediates(self.ctx, raw, rho)
        return decode_feat(raw, c.storage, c.K, c.H, c.W), rho

    def refocus(self, median=0):
        c = self.case
        rgb = np.zeros((c.H, c.W, 3), np.float32)
        d = np.zeros((c.H, c.W), np.int32)
        q = np.zeros((c.K, c.H, c.W), np.float32)
        hole = np.zeros((c.H, c.W), np.uint8)
        self.LF.lf_refocus(self.ctx, rgb, d, q, hole, median)
        return rgb, d, q, hole


# ---------------------------------------------------------------------------
# Comparisons
# ---------------------------------------------------------------------------

def near_tie(E1, E2):
    return (E2 - E1) <= NEAR_TIE * np.maximum(np.abs(E2), 1.0)


def rows_mask(H, W, rows):
    m = np.zeros((H, W), bool)
    y0, y1 = rows if rows is not None else (0, H)
    m[y0:y1] = True
    return m


def level_edge_exempt(case):
    """Pixels whose level set depends on a rounding of mu_T: a level within
    1e-4 of the search window's edge (the GPU tests |d - mu| <= window in
    single precision, the oracle in double).  The level nearest mu_T, which
    the variants fall back to, is formed in double on both sides (half-way
    goes to the lower level) and is not exempt."""
    mu = case.mu_T.astype(np.float64)
    ex = np.zeros(mu.shape, bool)
    if case.window > 0:
        for e in (mu - case.window, mu + case.window):
            te = (e - case.d_min) / case.d_step
            ex |= np.abs(te - np.rint(te)) < 1e-4
    return ex


def compare_iteration(case, ref, ref_soft, q_gpu, d_gpu, L_gpu, rows=None, label=""):
    """Compare one GPU iteration with the oracle's iteration from the same state.
    Returns a dict of statistics; raises AssertionError on a parity failure."""
    sel = rows_mask(case.H, case.W, rows)
    tie = near_tie(ref["E1"], ref["E2"]) & sel
    if case.flags:
        tie |= level_edge_exempt(case) & sel
    d_ok = (d_gpu == ref["d_idx"])
    bad_d = sel & ~d_ok & ~tie
    assert not bad_d.any(), f"{label}: d_idx differs off near-ties at {np.argwhere(bad_d)[:5].tolist()} " \
                            f"gpu={d_gpu[bad_d][:5]} oracle={ref['d_idx'][bad_d][:5]}"
    same = sel & d_ok
    qd = np.abs(q_gpu.astype(np.float64) - ref["q"])
    if case.mode == "enum_hard":
        # the arg max labeling is decided in FP32 on the GPU: exempt pixels
        # whose two largest labeling log weights are within 1e-3
        gap = enum_top_gap(case, ref["f"], ref["rho"], ref["omr"], ref["d_idx"], rows)
        decided = gap >= 1e-3
        bad_q = (qd > 0) & (decided & same)[None]
        assert not bad_q.any(), f"{label}: enumerated labels differ at {np.argwhere(bad_q)[:5].tolist()}"
    elif case.mode == "hard":
        z = np.log(np.clip(ref_soft["q"], 1e-300, 1.0)) - np.log(np.clip(1.0 - ref_soft["q"], 1e-300, 1.0))
        decided = np.abs(z) >= 1e-3
        bad_q = (qd > 0) & decided & same[None]
        assert not bad_q.any(), f"{label}: hard q differs at {np.argwhere(bad_q)[:5].tolist()}"
    else:
        qmax = float(qd[:, same].max()) if same.any() else 0.0
        assert qmax <= TOL_Q, f"{label}: q max-abs {qmax:.3g} > {TOL_Q}"
    # the objective's FP32 rounding error grows with the magnitude of its
    # addends (the log prior and each view's static and dynamic log weights),
    # which cancel in the sum: relative to that magnitude (never below |L|)
    if case.mode in ("soft", "hard") and "q_in" in ref:
        scale = objective_scale(case, ref["f"], ref["rho"], ref["omr"], ref["q_in"], ref["d_idx"], rows)
    else:
        scale = np.abs(ref["L"])
    Ld = np.abs(L_gpu.astype(np.float64) - ref["L"]) / np.maximum(scale, 1.0)
    Lmax = float(Ld[same].max()) if same.any() else 0.0
    assert Lmax <= TOL_L, f"{label}: objective rel diff {Lmax:.3g} > {TOL_L}"
    n = int(sel.sum())
    return {"pixels": n, "near_ties": int(tie.sum()), "d_mismatch_at_ties": int((sel & ~d_ok).sum()),
            "q_maxabs": float(qd[:, same].max()) if same.any() else 0.0, "L_maxrel": Lmax}


def objective_scale(case, f, rho, omr, q_in, d_idx, rows):
    """Per pixel, |ln prior(d)| + sum_k (max(|a1_k|, |a0_k|) + ln 2) at the
    oracle's level d, with a1_k = ln rho_k + lambda - beta/K |f_k - m|^2
    (m the M-step mean from the weights q_in) and a0_k = ln(1 - rho_k): the
    magnitude of the objective's addends (infinite log weights are exact on
    both sides and left out).  Never below |L|."""
    y0, y1 = rows if rows is not None else (0, case.H)
    K, W = case.K, case.W
    lam = O.lam_of(case.oracle_params())
    bp = case.beta / K
    out = np.zeros((case.H, W))
    xs = np.arange(W, dtype=np.float64)
    two_s2 = 2.0 * float(case.sigma) ** 2
    for y in range(y0, y1):
        d = case.d_min + d_idx[y].astype(np.float64) * case.d_step
        g = np.empty((K, W, 2))
        for k in range(K):
            for c in range(2):
                g[k, :, c] = np.interp(np.clip(xs - case.baselines[k] * d, 0, W - 1), xs, f[k, y, :, c])
        wt = q_in[:, y]
        Q = wt.sum(axis=0)
        wt = np.where(Q > 0, wt, 1.0)
        m = (wt[..., None] * g).sum(axis=0) / wt.sum(axis=0)[:, None]
        e = ((g - m[None]) ** 2).sum(axis=-1)
        with np.errstate(divide="ignore"):
            a1 = np.log(rho[:, y]) + lam - bp * e
            a0 = np.log(omr[:, y])
        fin = lambda a: np.where(np.isfinite(a), np.abs(a), 0.0)
        prior = np.log(case.gamma + np.exp(-(d - case.mu_T[y].astype(np.float64)) ** 2 / two_s2))
        out[y] = np.abs(prior) + (np.maximum(fin(a1), fin(a0)) + np.log(2.0)).sum(axis=0)
    return out


def enum_top_gap(case, f, rho, omr, d_idx, rows):
    """Gap between the two largest labeling log weights of the enumeration
    E-step at each pixel's level (used only to exempt near-ties)."""
    y0, y1 = rows if rows is not None else (0, case.H)
    K, W = case.K, case.W
    gap = np.full((case.H, W), np.inf)
    xs = np.arange(W, dtype=np.float64)
    for y in range(y0, y1):
        d = case.d_min + d_idx[y].astype(np.float64) * case.d_step
        g = np.empty((K, W, 2))
        for k in range(K):
            for c in range(2):
                g[k, :, c] = np.interp(xs - case.baselines[k] * d, np.arange(W, dtype=np.float64), f[k, y, :, c])
        with np.errstate(divide="ignore"):
            l1, l0 = np.log(rho[:, y]), np.log(omr[:, y])
        lws = []
        for mask in range(1 << K):
            S = np.array([(mask >> k) & 1 for k in range(K)], bool)
            lw = np.where(S[:, None], l1, l0).sum(axis=0)
            if S.sum() >= 2:
                lw = lw - case.beta * g[S].var(axis=0).sum(axis=-1)
            lws.append(lw)
        lws = np.sort(np.array(lws), axis=0)
        with np.errstate(invalid="ignore"):
            gap[y] = np.where(np.isfinite(lws[-2]), lws[-1] - lws[-2], np.inf)
    return gap


def teacher_forced(case: Case, n_iters: int, rows=None, device_inputs=True, check_refocus=True, q_warm=None,
                   expect=None):
    """Per-iteration parity of the GPU library against the oracle (see module doc).
    q_warm: first weights (a warm start) instead of the threshold.  expect:
    (rgb, d_idx, q) another GPU path produced for the same frame, which must
    equal this chain's final state bit for bit on the whole frame."""
    op = case.oracle_params()
    y0, y1 = rows if rows is not None else (0, case.H)
    orows = (max(0, y0 - 1), min(case.H, y1 + 1))
    f_o = O.descriptors(op, case.views, rows=orows)
    pr = O.ray_prior(op, case.S_P, case.mu_T, rows=(y0, y1))
    rho_o, q0_o = pr
    omr_o = pr.omr
    run = DeviceRun(case, device_inputs=device_inputs, q_warm=q_warm)
    try:
        f_g, rho_g = run.intermediates()
        assert np.array_equal(f_g[:, y0:y1], f_o[:, y0:y1]), "descriptors differ"
        rdiff = np.abs(rho_g[:, y0:y1].astype(np.float64) - rho_o[:, y0:y1]).max()
        assert rdiff <= TOL_RHO, f"rho max-abs {rdiff:.3g}"
        q_prev, _, _ = run.state(with_d=False)
        if q_warm is not None:
            assert np.array_equal(q_prev, np.asarray(q_warm, np.float32)), "warm start not taken as given"
        else:
            near_tau = np.abs(rho_o - case.tau) < 1e-6
            bad = (q_prev[:, y0:y1] != q0_o[:, y0:y1]) & ~near_tau[:, y0:y1]
            assert not bad.any(), "first weights differ off the threshold"
        stats = []
        for t in range(n_iters):
            run.iterate(1)
            q_g, d_g, L_g = run.state()
            ref = O.em_iteration(op, f_o, rho_o, case.mu_T, q_prev.astype(np.float64), rows=(y0, y1), omr=omr_o)
            ref.update(f=f_o, rho=rho_o, omr=omr_o, q_in=q_prev.astype(np.float64))
            ref_soft = ref
            if case.mode == "hard":
                ref_soft = O.em_iteration(case.oracle_params(mode="soft"), f_o, rho_o, case.mu_T,
                                          q_prev.astype(np.float64), rows=(y0, y1), omr=omr_o)
            stats.append(compare_iteration(case, ref, ref_soft, q_g, d_g, L_g, rows=(y0, y1), label=f"iter {t + 1}"))
            q_prev = q_g
        if check_refocus and n_iters > 0:
            rgb_g, d_g, q_g, hole_g = run.refocus()
            rgb_o, hole_o = O.refocus(op, case.views, d_g, q_g.astype(np.float64), rows=(y0, y1), rho=rho_o)
            assert np.array_equal(hole_g[y0:y1], hole_o[y0:y1]), "hole mask differs"
            near_half = (np.abs(q_g.astype(np.float64) - 0.5) < 1e-4).any(axis=0)
            cmp = ~near_half[y0:y1]
            rd = np.abs(rgb_g[y0:y1].astype(np.float64) - rgb_o[y0:y1]).max(axis=-1)
            rmax = float(rd[cmp].max()) if cmp.any() else 0.0
            assert rmax <= TOL_RGB, f"refocus max-abs {rmax:.3g}"
            stats.append({"refocus_maxabs": rmax})
            if expect is not None:
                for name, a, b in zip(("rgb", "d_idx", "q"), expect, (rgb_g, d_g, q_g)):
                    a = np.asarray(a)
                    bad = np.argwhere(a != b)
                    assert not len(bad), f"{name} differs from the other path's at {len(bad)} places, " \
                                         f"first {bad[:3].tolist()}: {a[tuple(bad[0])]} vs {b[tuple(bad[0])]}"
        return stats
    finally:
        run.close()


# ---------------------------------------------------------------------------
# Workload frames and row bands
# ---------------------------------------------------------------------------

_FRAMES = {}


def workload_frame(name):
    """The workload's seeded frame, generated once per test session."""
    import lf_scenes as S
    if name not in _FRAMES:
        _FRAMES[name] = S.make_frame(S.workload_spec(name))
    return _FRAMES[name]


def row_bands(case, n=8):
    """Four bands of n rows: the top edge, the bottom edge, the band whose
    reference rays are most often dynamic by the threshold (through a moving
    object), and the middle of the frame."""
    H = case.H
    n = min(n, H)
    dyn = (case.S_P[case.ref] < case.tau).mean(axis=1)
    run = np.convolve(dyn, np.ones(n), mode="valid")
    yd = int(np.argmax(run))
    ym = max(0, min(H - n, H // 2 - n // 2))
    bands = [(0, n), (H - n, H), (yd, yd + n), (ym, ym + n)]
    out = []
    for b in bands:
        if b not in out:
            out.append(b)
    return out
