"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
library routine (scipy's Sobel, numpy's interp/var/float16, torch's bfloat16,
scipy's Gaussian density), a closed form, a brute-force enumeration of all
segmentation labelings, or an invariant EM guarantees.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(20260)


def _params(K, H, W, b, D, beta, ref=None, d_min=0.0, d_step=1.0, **kw):
    ref = ref if ref is not None else int(np.argmin(np.abs(np.asarray(b))))
    return O.make_params(K, H, W, ref, b, d_min, d_step, D, beta, **kw)


def _random_views(K, H, W, rng=RNG):
    return rng.integers(0, 256, size=(K, H, W, 3), dtype=np.uint8)


def _interp_row(row, u):
    """Linear interpolation with end clamping (numpy's interp)."""
    return np.interp(u, np.arange(row.shape[0], dtype=np.float64), row)


def _gathered(f, b, y, x, d):
    """[K][2] descriptors of reference pixel (x, y) at disparity d, via np.interp."""
    K = f.shape[0]
    return np.array([[_interp_row(f[k, y, :, c], x - b[k] * d) for c in range(2)] for k in range(K)])


# ---------------------------------------------------------------- storage rounding

def test_round_fp16_matches_numpy():
    vals = np.concatenate([
        RNG.uniform(-1, 1, 4000),
        RNG.uniform(0, 1e-4, 500),                      # subnormal range of binary16
        np.arange(-3060, 3061) / 4096.0,                # every possible descriptor value
        (np.arange(2049, 4096, 2) + 0.5) / 4096.0,      # exact ties
    ])
    ours = np.array([O.round_storage(v, "f16") for v in vals])
    ref = vals.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    vals = np.concatenate([
        RNG.uniform(-1, 1, 4000).astype(np.float32),
        (np.arange(-3060, 3061) / 4096.0).astype(np.float32),
        np.float32(1.0) + np.arange(0, 64).astype(np.float32) * np.float32(2.0 ** -9),  # ties at 1.x
        RNG.uniform(0, 1, 500).astype(np.float32),
    ]).astype(np.float32)
    ours = np.array([O.round_storage(float(v), "bf16") for v in vals])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


# ---------------------------------------------------------------- descriptors

def test_descriptors_match_scipy_sobel():
    from scipy.ndimage import sobel
    K, H, W = 3, 17, 23
    views = _random_views(K, H, W)
    p = _params(K, H, W, [-1, 0, 1], 4, 100.0)
    f = O.descriptors(p, views)
    for k in range(K):
        L = views[k].astype(np.float64).sum(axis=2)
        gx = sobel(L, axis=1, mode="nearest") / 4096.0
        gy = sobel(L, axis=0, mode="nearest") / 4096.0
        assert np.array_equal(f[k, :, :, 0], gx)
        assert np.array_equal(f[k, :, :, 1], gy)


def test_descriptors_linear_ramp():
    # L = a x + c y  =>  Gx = 8a, Gy = 8c away from the border (textbook Sobel)
    H, W, a, c = 12, 20, 3, 5
    y, x = np.mgrid[0:H, 0:W]
    L = a * x + c * y
    views = np.zeros((2, H, W, 3), np.uint8)
    views[:, :, :, 0] = np.minimum(L, 255)
    views[:, :, :, 1] = np.clip(L - 255, 0, 255)
    assert L.max() <= 510
    p = _params(2, H, W, [0, 1], 4, 100.0)
    f = O.descriptors(p, views)
    assert np.all(f[0, 1:-1, 1:-1, 0] * 4096 == 8 * a)
    assert np.all(f[0, 1:-1, 1:-1, 1] * 4096 == 8 * c)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_descriptors_mirrored_rounding(storage):
    torch = pytest.importorskip("torch")
    K, H, W = 2, 9, 31
    # high-contrast columns: many |G| above 2048, where binary16 must round
    hi = RNG.integers(0, 2, size=(K, 1, W, 1)) * 235
    views = (hi + RNG.integers(0, 21, size=(K, H, W, 3))).astype(np.uint8)
    exact = O.descriptors(_params(K, H, W, [0, 1], 4, 100.0), views)
    low = O.descriptors(_params(K, H, W, [0, 1], 4, 100.0, storage=storage), views)
    if storage == "f16":
        ref = exact.astype(np.float16).astype(np.float64)
    else:
        ref = torch.from_numpy(exact.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(low, ref)
    assert not np.array_equal(low, exact)      # the rounding is really applied


# ---------------------------------------------------------------- ray prior

@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_ray_prior_is_interp_of_SP(storage):
    K, H, W = 3, 6, 40
    b = [-1.5, 0.0, 2.0]
    S_P = RNG.uniform(0, 1, (K, H, W)).astype(np.float32)
    mu = RNG.uniform(-3, 12, (H, W)).astype(np.float32)
    p = _params(K, H, W, b, 8, 100.0, ref=1, storage=storage)
    pr = O.ray_prior(p, S_P, mu)
    rho, q0 = pr
    sp = S_P.astype(np.float16).astype(np.float64) if storage == "f16" else S_P.astype(np.float64)
    for k in range(K):
        for y in range(H):
            u = np.arange(W) - b[k] * mu[y].astype(np.float64)
            np.testing.assert_allclose(rho[k, y], _interp_row(sp[k, y], u), rtol=0, atol=1e-15)
            np.testing.assert_allclose(pr.omr[k, y], _interp_row(1.0 - sp[k, y], u), rtol=1e-14, atol=0)
    assert np.array_equal(q0, (rho >= 0.7).astype(np.float64))


# ---------------------------------------------------------------- likelihood constant

def test_lambda_is_gaussian_over_uniform_density():
    from scipy.stats import multivariate_normal
    for K, beta in [(5, 2133.0), (9, 75000.0), (3, 10.0)]:
        p = _params(K, 4, 4, list(range(K)), 4, beta, ref=0)
        bp = beta / K
        gauss_peak = multivariate_normal(mean=[0, 0], cov=np.eye(2) / (2 * bp)).pdf([0, 0])
        uniform = 1.0 / (2 * 3060 / 4096) ** 2
        assert math.isclose(O.derive_lambda(p), math.log(gauss_peak / uniform), rel_tol=1e-12)


# ---------------------------------------------------------------- M-step

def _energies_from_variance(f, b, y, x, levels, beta, gamma, sigma, mu):
    """All-static energies: beta * (population variance over views, summed over features)."""
    E = []
    for d in levels:
        g = _gathered(f, b, y, x, d)
        var = np.var(g, axis=0).sum()
        E.append(beta * var + math.log1p(gamma) - math.log(gamma + math.exp(-(d - mu) ** 2 / (2 * sigma ** 2))))
    return np.array(E)


@pytest.mark.parametrize("d_step", [1.0, 0.5, 0.75])
def test_mstep_all_static_is_beta_times_variance(d_step):
    K, H, W, D = 4, 5, 30, 9
    b = [0.0, 1.0, 2.0, -1.0]
    views = _random_views(K, H, W)
    mu = RNG.uniform(0, 6, (H, W)).astype(np.float32)
    p = _params(K, H, W, b, D, 300.0, ref=0, d_min=-1.0, d_step=d_step)
    f = O.descriptors(p, views)
    rho = np.ones((K, H, W))
    out = O.em_iteration(p, f, rho, mu, np.ones((K, H, W)))
    levels = -1.0 + d_step * np.arange(D)
    for y in range(H):
        for x in range(W):
            E = _energies_from_variance(f, b, y, x, levels, 300.0, 0.05, 2.0, float(mu[y, x]))
            assert out["d_idx"][y, x] == int(np.argmin(E))
            srt = np.sort(E)
            assert math.isclose(out["E1"][y, x], srt[0], rel_tol=1e-11, abs_tol=1e-11)
            assert math.isclose(out["E2"][y, x], srt[1], rel_tol=1e-11, abs_tol=1e-11)


def test_mstep_weighted_matches_pairwise_form():
    # sum_k q_k |f_k - m|^2 = (1/2Q) sum_k sum_l q_k q_l |f_k - f_l|^2
    K, H, W, D = 5, 4, 26, 7
    b = [-2.0, -1.0, 0.0, 1.0, 2.0]
    views = _random_views(K, H, W)
    mu = RNG.uniform(0, 6, (H, W)).astype(np.float32)
    q = RNG.uniform(0, 1, (K, H, W))
    q[:, 0, :3] = 0.0                       # no weight at all: the prior decides
    beta, gamma, sigma = 800.0, 0.05, 2.0
    p = _params(K, H, W, b, D, beta, ref=2)
    f = O.descriptors(p, views)
    out = O.em_iteration(p, f, np.full((K, H, W), 0.5), mu, q)
    for y in range(H):
        for x in range(W):
            E = []
            for j in range(D):
                g = _gathered(f, b, y, x, float(j))
                w = q[:, y, x]
                Q = w.sum()
                diff = ((g[:, None, :] - g[None, :, :]) ** 2).sum(-1)
                C = (w[:, None] * w[None, :] * diff).sum() / (2 * Q) if Q > 0 else 0.0
                E.append(beta / K * C + math.log1p(gamma)
                         - math.log(gamma + math.exp(-(j - float(mu[y, x])) ** 2 / (2 * sigma ** 2))))
            E = np.array(E)
            assert out["d_idx"][y, x] == int(np.argmin(E))
            assert math.isclose(out["E1"][y, x], E.min(), rel_tol=1e-10, abs_tol=1e-10)


def test_mstep_beta_zero_picks_level_nearest_prior():
    K, H, W, D = 3, 4, 20, 16
    views = _random_views(K, H, W)
    mu = RNG.uniform(-2, 10, (H, W)).astype(np.float32)
    mu[0, 0] = 2.25    # exact tie between levels 2.0 and 2.5 -> the lower level
    p = _params(K, H, W, [0, 1, 2], D, 0.0, ref=0, lam=0.0, d_min=-1.0, d_step=0.5)
    f = O.descriptors(p, views)
    out = O.em_iteration(p, f, np.full((K, H, W), 0.5), mu, RNG.uniform(0, 1, (K, H, W)))
    levels = -1.0 + 0.5 * np.arange(D)
    want = np.argmin(np.abs(levels[None, None, :] - mu[..., None].astype(np.float64)), axis=-1)
    assert np.array_equal(out["d_idx"], want)
    assert out["d_idx"][0, 0] == 6


def test_mstep_recovers_fronto_parallel_plane():
    # a textured plane at integer disparity d0, asymmetric baselines: the sign
    # and scale of the shift are fixed by recovering d0 exactly
    K, H, W, D, d0 = 3, 10, 80, 12, 5
    b = [0.0, 1.0, 3.0]
    rng = np.random.default_rng(7)
    tex = rng.integers(0, 256, size=(H, W + 3 * D + 2, 3), dtype=np.uint8)
    views = np.empty((K, H, W, 3), np.uint8)
    xs = np.arange(W)
    for k in range(K):
        views[k] = tex[:, xs + int(b[k] * d0)]      # view k pixel x sees u = x + b_k d0
    mu = np.full((H, W), 6.0, np.float32)           # prior off by one level
    p = _params(K, H, W, b, D, 2133.0, ref=0, sigma=4.0)
    f = O.descriptors(p, views)
    out = O.em_iteration(p, f, np.ones((K, H, W)), mu, np.ones((K, H, W)))
    # view k samples x - b_k d: columns below 3*d0 (+1 for the Sobel) fall outside view 3
    assert np.all(out["d_idx"][:, 3 * d0 + 1:W - 1] == d0)


# ---------------------------------------------------------------- E-step

def _enumerate(rho, lam, bp, e):
    """Joint over all 2^K labelings: marginals P(S_k=1), MAP labeling, log sum, log max."""
    K = len(rho)
    tot, best, best_S = 0.0, -1.0, None
    marg = np.zeros(K)
    for S in itertools.product([0, 1], repeat=K):
        p = 1.0
        for k in range(K):
            p *= rho[k] * math.exp(lam - bp * e[k]) if S[k] else (1.0 - rho[k])
        tot += p
        marg += p * np.array(S)
        if p > best:
            best, best_S = p, S
    return marg / tot, np.array(best_S, float), math.log(tot), math.log(best)


@pytest.mark.parametrize("mode", ["soft", "hard"])
def test_estep_and_objective_match_enumeration(mode):
    K, H, W, D = 4, 3, 18, 6
    b = [-1.0, 0.0, 1.0, 2.0]
    views = _random_views(K, H, W)
    mu = RNG.uniform(0, 5, (H, W)).astype(np.float32)
    beta, lam, gamma, sigma = 60.0, 1.3, 0.05, 2.0
    p = _params(K, H, W, b, D, beta, ref=1, lam=lam, mode=mode)
    f = O.descriptors(p, views)
    rho = RNG.uniform(0.02, 0.98, (K, H, W))
    q_in = RNG.uniform(0, 1, (K, H, W))
    out = O.em_iteration(p, f, rho, mu, q_in)
    for y in range(H):
        for x in range(W):
            d = float(out["d_idx"][y, x])
            g = _gathered(f, b, y, x, d)
            m = np.average(g, axis=0, weights=q_in[:, y, x])
            e = ((g - m) ** 2).sum(axis=1)
            marg, S_map, log_sum, log_max = _enumerate(rho[:, y, x], lam, beta / K, e)
            prior = math.log(gamma + math.exp(-(d - float(mu[y, x])) ** 2 / (2 * sigma ** 2)))
            if mode == "soft":
                np.testing.assert_allclose(out["q"][:, y, x], marg, rtol=1e-11, atol=1e-13)
                assert math.isclose(out["L"][y, x], prior + log_sum, rel_tol=1e-11)
            else:
                assert np.array_equal(out["q"][:, y, x], S_map)
                assert math.isclose(out["L"][y, x], prior + log_max, rel_tol=1e-11)


def test_estep_certain_priors_are_kept():
    K, H, W = 3, 2, 10
    views = _random_views(K, H, W)
    p = _params(K, H, W, [0, 1, 2], 5, 500.0, ref=0)
    f = O.descriptors(p, views)
    rho = RNG.integers(0, 2, (K, H, W)).astype(np.float64)
    rho[:, 0, 0] = 0.0                       # no static view at all
    out = O.em_iteration(p, f, rho, np.zeros((H, W), np.float32), np.ones((K, H, W)))
    assert np.array_equal(out["q"], rho)
    assert np.all(np.isfinite(out["L"]))


def test_estep_beta_zero_is_logistic_prior():
    from scipy.special import expit, logit
    K, H, W = 3, 3, 12
    views = _random_views(K, H, W)
    lam = 0.7
    p = _params(K, H, W, [0, 1, 2], 5, 0.0, ref=0, lam=lam)
    f = O.descriptors(p, views)
    rho = RNG.uniform(0.01, 0.99, (K, H, W))
    out = O.em_iteration(p, f, rho, np.zeros((H, W), np.float32), np.ones((K, H, W)))
    np.testing.assert_allclose(out["q"], expit(logit(rho) + lam), rtol=1e-12)


# ---------------------------------------------------------------- enumeration E-step

def _enum_case(K, H, W, b, beta, mode, rng, rho_lo=0.02, rho_hi=0.98, views=None):
    views = _random_views(K, H, W, rng) if views is None else views
    mu = rng.uniform(0, 4, (H, W)).astype(np.float32)
    p = _params(K, H, W, b, 6, beta, mode=mode)
    f = O.descriptors(p, views)
    rho = rng.uniform(rho_lo, rho_hi, (K, H, W))
    q_in = rng.uniform(0, 1, (K, H, W))
    return p, f, rho, mu, q_in, O.em_iteration(p, f, rho, mu, q_in)


@pytest.mark.parametrize("mode", ["enum_soft", "enum_hard"])
def test_enum_two_views_closed_form(mode):
    """K = 2: only the labeling with both views static has a variance, and
    the population variance of two vectors is a quarter of their squared
    distance; the other three labelings weigh by their priors alone."""
    rng = np.random.default_rng(41)
    beta = 40.0
    p, f, rho, mu, q_in, out = _enum_case(2, 3, 14, [0.0, 1.0], beta, mode, rng)
    for y in range(3):
        for x in range(14):
            d = float(out["d_idx"][y, x])
            g = _gathered(f, [0.0, 1.0], y, x, d)
            r1, r2 = rho[0, y, x], rho[1, y, x]
            w11 = r1 * r2 * math.exp(-beta * float(((g[0] - g[1]) ** 2).sum()) / 4.0)
            w10, w01, w00 = r1 * (1 - r2), (1 - r1) * r2, (1 - r1) * (1 - r2)
            Z = w11 + w10 + w01 + w00
            prior = math.log(p.gamma + math.exp(-(d - float(mu[y, x])) ** 2 / (2 * p.sigma ** 2)))
            if mode == "enum_soft":
                np.testing.assert_allclose(out["q"][:, y, x], [(w11 + w10) / Z, (w11 + w01) / Z], rtol=1e-12)
                assert math.isclose(out["L"][y, x], prior + math.log(Z), rel_tol=1e-12)
            else:
                ws = {(1, 1): w11, (1, 0): w10, (0, 1): w01, (0, 0): w00}
                best = max(ws, key=ws.get)
                assert tuple(out["q"][:, y, x]) == best
                assert math.isclose(out["L"][y, x], prior + math.log(ws[best]), rel_tol=1e-12)


def test_enum_matches_brute_force_with_numpy_var():
    """K = 4: marginals and the arg max of the joint over all 16 labelings,
    weighted by exp(-beta numpy.var(static descriptors)) and the priors."""
    rng = np.random.default_rng(42)
    b = [-1.0, 0.0, 1.0, 2.0]
    beta = 25.0
    for mode in ("enum_soft", "enum_hard"):
        p, f, rho, mu, q_in, out = _enum_case(4, 2, 12, b, beta, mode, rng)
        for y in range(2):
            for x in range(12):
                g = _gathered(f, b, y, x, float(out["d_idx"][y, x]))
                marg, tot, best, best_S = np.zeros(4), 0.0, -1.0, None
                for S in itertools.product([0, 1], repeat=4):
                    Sa = np.array(S, bool)
                    var = float(np.var(g[Sa], axis=0).sum()) if Sa.sum() >= 2 else 0.0
                    w = math.exp(-beta * var) * float(np.prod(np.where(Sa, rho[:, y, x], 1 - rho[:, y, x])))
                    tot += w
                    marg += w * Sa
                    if w > best:
                        best, best_S = w, Sa
                if mode == "enum_soft":
                    np.testing.assert_allclose(out["q"][:, y, x], marg / tot, rtol=1e-11, atol=1e-14)
                else:
                    assert np.array_equal(out["q"][:, y, x], best_S.astype(float))


def test_enum_beta_zero_and_certain_priors():
    rng = np.random.default_rng(43)
    b = [-1.0, 0.0, 1.0]
    # beta = 0: the labels are independent, the marginal is the prior
    _, _, rho, _, _, out = _enum_case(3, 2, 10, b, 0.0, "enum_soft", rng)
    np.testing.assert_allclose(out["q"], rho, rtol=1e-12)
    _, _, rho, _, _, out = _enum_case(3, 2, 10, b, 0.0, "enum_hard", rng)
    assert np.array_equal(out["q"], (rho >= 0.5).astype(float))
    # every labeling ties at rho = 1/2: the tie goes to the largest mask (all static)
    _, _, _, _, _, out = _enum_case(3, 2, 10, b, 0.0, "enum_hard", rng, rho_lo=0.5, rho_hi=0.5)
    assert np.all(out["q"] == 1.0)
    # certain priors stay certain whatever the descriptors say
    for mode in ("enum_soft", "enum_hard"):
        p, f, _, mu, q_in, _ = _enum_case(3, 2, 10, b, 300.0, mode, rng)
        rho = rng.integers(0, 2, (3, 2, 10)).astype(np.float64)
        out = O.em_iteration(p, f, rho, mu, q_in)
        assert np.array_equal(out["q"], rho)


def test_enum_identical_views_weigh_by_prior_only():
    """Every view shows the same colours: every variance is zero, so the
    enumeration returns the prior whatever beta is."""
    rng = np.random.default_rng(44)
    one = _random_views(1, 3, 16, rng)
    views = np.repeat(one, 4, axis=0)
    _, _, rho, _, _, out = _enum_case(4, 3, 16, [0.0, 0.0, 0.0, 0.0], 500.0, "enum_soft", rng, views=views)
    np.testing.assert_allclose(out["q"], rho, rtol=1e-12)


def test_enum_mstep_is_the_weighted_sweep():
    """The enumeration modes change the E-step only: the M-step level is the
    one of the factorised modes for the same weights."""
    rng = np.random.default_rng(45)
    K, H, W = 4, 3, 20
    views = _random_views(K, H, W, rng)
    b = [-1.0, 0.0, 1.0, 2.0]
    mu = rng.uniform(0, 4, (H, W)).astype(np.float32)
    rho = rng.uniform(0.05, 0.95, (K, H, W))
    q_in = rng.uniform(0, 1, (K, H, W))
    d = {}
    for mode in ("soft", "enum_soft", "enum_hard"):
        p = _params(K, H, W, b, 6, 80.0, mode=mode)
        d[mode] = O.em_iteration(p, O.descriptors(p, views), rho, mu, q_in)["d_idx"]
    assert np.array_equal(d["soft"], d["enum_soft"]) and np.array_equal(d["soft"], d["enum_hard"])


# ---------------------------------------------------------------- work-avoiding variants

@pytest.mark.parametrize("window", [1.5, 3.0, 6.0])
def test_window_sweep_is_arg_min_over_levels_near_prior(window):
    """The windowed M-step is the arg min of the all-static energies
    (beta numpy.var form) over the levels with |d - mu| <= window, and the
    level nearest mu when no level is that close."""
    K, H, W, D = 4, 4, 24, 12
    b = [0.0, 1.0, 2.0, -1.0]
    views = _random_views(K, H, W)
    mu = RNG.uniform(-1, 7, (H, W)).astype(np.float32)
    mu[0, :4] = [-9.0, 30.0, 5.001, 5.0]      # two empty windows; levels exactly at the window edge
    d_min, d_step = -1.0, 0.75
    p = _params(K, H, W, b, D, 300.0, ref=0, d_min=d_min, d_step=d_step, window=window)
    f = O.descriptors(p, views)
    out = O.em_iteration(p, f, np.ones((K, H, W)), mu, np.ones((K, H, W)))
    levels = d_min + d_step * np.arange(D)
    for y in range(H):
        for x in range(W):
            m = float(mu[y, x])
            inside = np.abs(levels - m) <= window
            E = _energies_from_variance(f, b, y, x, levels, 300.0, 0.05, 2.0, m)
            if inside.any():
                want = int(np.flatnonzero(inside)[np.argmin(E[inside])])
            else:
                want = int(np.argmin(np.abs(levels - m)))
            assert out["d_idx"][y, x] == want, (y, x)


def test_window_edge_levels_are_searched():
    """A level exactly `window` away from mu is inside the window: with mu
    half-way between two levels and window half a step, both are searched."""
    K, H, W, D = 4, 2, 30, 12
    b = [0.0, 1.0, 2.0, -1.0]
    views = _random_views(K, H, W)
    mu = np.full((H, W), 5.375, np.float32)          # between levels 8 (5.0) and 9 (5.75)
    p = _params(K, H, W, b, D, 300.0, ref=0, d_min=-1.0, d_step=0.75, window=0.375)
    f = O.descriptors(p, views)
    out = O.em_iteration(p, f, np.ones((K, H, W)), mu, np.ones((K, H, W)))
    levels = -1.0 + 0.75 * np.arange(D)
    for y in range(H):
        for x in range(W):
            E = _energies_from_variance(f, b, y, x, levels[8:10], 300.0, 0.05, 2.0, 5.375)
            assert out["d_idx"][y, x] == 8 + int(np.argmin(E))
    assert (out["d_idx"] == 9).any()


def test_window_covering_every_level_is_the_full_sweep():
    K, H, W, D = 3, 3, 20, 10
    views = _random_views(K, H, W)
    mu = RNG.uniform(0, 9, (H, W)).astype(np.float32)
    q = RNG.uniform(0, 1, (K, H, W))
    rho = RNG.uniform(0.1, 0.9, (K, H, W))
    outs = []
    for window in (0.0, 100.0):
        p = _params(K, H, W, [-1, 0, 1], D, 500.0, ref=1, window=window)
        outs.append(O.em_iteration(p, O.descriptors(p, views), rho, mu, q))
    for key in ("q", "d_idx", "L"):
        assert np.array_equal(outs[0][key], outs[1][key])


def test_dynamic_only_reconstructs_exactly_the_dynamic_reference_pixels():
    """dyn_only: pixels whose reference ray is dynamic by the prior threshold
    get the results of the full method; the others keep their weights, the
    level nearest mu, no objective, and their reference colour."""
    rng = np.random.default_rng(46)
    K, H, W, D = 5, 6, 40, 12
    b = [-2.0, -1.0, 0.0, 1.0, 2.0]
    views = rng.integers(0, 256, size=(K, H, W, 3), dtype=np.uint8)
    S_P = rng.uniform(0, 1, (K, H, W)).astype(np.float32)
    tau = float(np.float32(0.7))
    S_P[2, 0, :5] = tau                      # exactly tau: static
    mu = rng.uniform(0, 11, (H, W)).astype(np.float32)
    res = {}
    for dyn in (False, True):
        p = _params(K, H, W, b, D, 400.0, ref=2, dyn_only=dyn, tau=tau)
        res[dyn] = O.reconstruct(p, views, S_P, mu, 3)
    rho_ref = res[True]["rho"][2]
    dyn = rho_ref < tau
    assert dyn.any() and (~dyn).any() and not dyn[0, :5].any()
    full, part = res[False], res[True]
    assert np.array_equal(part["d_idx"][dyn], full["d_idx"][dyn])
    assert np.array_equal(part["q"][:, dyn], full["q"][:, dyn])
    assert np.array_equal(part["rgb"][dyn], full["rgb"][dyn])
    assert np.array_equal(part["hole"][dyn], full["hole"][dyn])
    levels = np.arange(D, dtype=np.float64)
    nearest = np.argmin(np.abs(levels[None, None, :] - mu[..., None].astype(np.float64)), axis=-1)
    assert np.array_equal(part["d_idx"][~dyn], nearest[~dyn])
    p = _params(K, H, W, b, D, 400.0, ref=2, tau=tau)
    _, q0 = O.ray_prior(p, S_P, mu)
    assert np.array_equal(part["q"][:, ~dyn], q0[:, ~dyn])
    assert np.all(part["L"][~dyn] == 0.0)
    assert np.array_equal(part["rgb"][~dyn], views[2][~dyn] / 255.0)
    assert not part["hole"][~dyn].any()


# ---------------------------------------------------------------- EM loop

@pytest.mark.parametrize("mode", ["soft", "hard"])
def test_em_objective_never_decreases(mode):
    K, H, W, D = 5, 12, 48, 16
    rng = np.random.default_rng(3)
    views = rng.integers(0, 256, size=(K, H, W, 3), dtype=np.uint8)
    S_P = rng.uniform(0, 1, (K, H, W)).astype(np.float32)
    mu = rng.uniform(0, 15, (H, W)).astype(np.float32)
    p = _params(K, H, W, [-2, -1, 0, 1, 2], D, 500.0, ref=2, mode=mode)
    f = O.descriptors(p, views)
    rho, q = O.ray_prior(p, S_P, mu)
    prev = None
    for t in range(6):
        out = O.em_iteration(p, f, rho, mu, q)
        if prev is not None:
            assert np.all(out["L"] >= prev - 1e-9 * np.maximum(1.0, np.abs(prev)))
        prev, q = out["L"], out["q"]
        assert np.all((q >= 0) & (q <= 1))


# ---------------------------------------------------------------- refocus

def test_refocus_all_static_is_plain_mean():
    K, H, W = 4, 5, 25
    b = [0.0, 1.0, -1.0, 2.5]
    views = _random_views(K, H, W)
    p = _params(K, H, W, b, 10, 100.0, ref=0, d_step=0.5)
    d_idx = RNG.integers(0, 10, (H, W)).astype(np.int32)
    rgb, hole = O.refocus(p, views, d_idx, np.ones((K, H, W)))
    assert not hole.any()
    for y in range(H):
        for x in range(W):
            d = 0.5 * d_idx[y, x]
            want = np.mean([[_interp_row(views[k, y, :, c].astype(float), x - b[k] * d) for c in range(3)]
                            for k in range(K)], axis=0) / 255.0
            np.testing.assert_allclose(rgb[y, x], want, rtol=0, atol=1e-14)


def test_refocus_one_none_and_half():
    K, H, W = 3, 2, 9
    views = _random_views(K, H, W)
    p = _params(K, H, W, [0.0, 1.0, 2.0], 4, 100.0, ref=0)
    d_idx = np.full((H, W), 1, np.int32)
    q = np.zeros((K, H, W))
    q[2, 0, :] = 0.5                          # exactly 0.5 counts as static
    rgb, hole = O.refocus(p, views, d_idx, q)
    for x in range(W):
        assert np.array_equal(rgb[0, x], views[2, 0, max(x - 2, 0)] / 255.0)
        assert hole[0, x] == 0
        assert np.array_equal(rgb[1, x], views[0, 1, x] / 255.0)   # none static: reference pixel
        assert hole[1, x] == 1


def test_threshold_start_counts_tau_as_static():
    # S_P exactly at tau at integer footprints: the ray starts static (S_P >= tau)
    K, H, W = 3, 2, 12
    S_P = np.full((K, H, W), 0.5, np.float32)
    S_P[:, 1, :] = np.nextafter(np.float32(0.5), np.float32(0))
    p = _params(K, H, W, [0, 1, 2], 4, 100.0, ref=0, tau=0.5)
    rho, q0 = O.ray_prior(p, S_P, np.full((H, W), 2.0, np.float32))
    assert np.all(q0[:, 0] == 1.0) and np.all(q0[:, 1] == 0.0)


def test_hard_assignment_tie_is_static():
    # identical flat views: e_k = 0; rho = 1/2 and lambda = 0 make a1 == a0
    K, H, W = 3, 2, 8
    views = np.full((K, H, W, 3), 100, np.uint8)
    p = _params(K, H, W, [0, 1, 2], 4, 100.0, ref=0, lam=0.0, mode="hard")
    f = O.descriptors(p, views)
    out = O.em_iteration(p, f, np.full((K, H, W), 0.5), np.zeros((H, W), np.float32), np.ones((K, H, W)))
    assert np.all(out["q"] == 1.0)
    np.testing.assert_allclose(out["L"], math.log(1.05) + K * math.log(0.5), rtol=1e-14)


def test_median3_matches_scipy():
    from scipy.ndimage import median_filter
    H, W = 9, 14
    p = _params(2, H, W, [0, 1], 4, 100.0, ref=0)
    rgb = RNG.uniform(0, 1, (H, W, 3))
    rgb[2, 3] = rgb[2, 4]                      # repeated values
    out = O.median3(p, rgb)
    for c in range(3):
        assert np.array_equal(out[:, :, c], median_filter(rgb[:, :, c], size=3, mode="nearest"))


def test_dynamic_prior_keeps_relative_accuracy_near_certainty():
    # rho within 1e-12 of 1: omr carries the dynamic prior to full relative
    # precision (the E-step takes its logarithm)
    K, H, W = 2, 1, 4
    S_P = np.array([[[1.0, np.float32(1.0 - 2 ** -20), 1.0, 1.0]], [[0.5] * 4]], np.float32)
    mu = np.full((H, W), 1e-6, np.float32)
    p = _params(K, H, W, [0.0, 1.0], 4, 100.0, ref=0)
    pr = O.ray_prior(p, np.ascontiguousarray(S_P[[1, 0]]), mu)
    u = 2 - 1.0 * np.float64(np.float32(1e-6))          # view 1, pixel 2: just left of column 2
    t = u - np.floor(u)
    want = (1 - t) * 2.0 ** -20                          # interpolation of 1 - S_P between columns 1 and 2
    assert abs(pr.omr[1, 0, 2] - want) <= 1e-12 * want
    assert pr.omr[1, 0, 3] == 0.0 and pr[0][1, 0, 3] == 1.0   # exact certainty stays exact


# ---------------------------------------------------------------- per-view segmentation maps

def test_segmentation_reference_view_is_identity():
    rng = np.random.default_rng(50)
    K, H, W, D = 3, 4, 20, 8
    p = _params(K, H, W, [-1.0, 0.0, 1.5], D, 100.0, ref=1)
    d = rng.integers(0, D, (H, W)).astype(np.int32)
    q = rng.uniform(0, 1, (K, H, W))
    lab = O.segmentation_maps(p, d, q)
    assert np.array_equal(lab[1], (q[1] >= 0.5).astype(np.uint8))


def test_segmentation_constant_level_is_a_shift():
    """All pixels at one level: view k's pixel u shows reference pixel
    u + b_k d (integer shift), nothing beyond the frame edge."""
    rng = np.random.default_rng(51)
    K, H, W, D, j0 = 4, 3, 25, 6, 3
    b = [-2.0, 0.0, 1.0, 3.0]
    p = _params(K, H, W, b, D, 100.0, ref=1, d_min=0.0, d_step=1.0)
    d = np.full((H, W), j0, np.int32)
    q = rng.uniform(0, 1, (K, H, W))
    lab = O.segmentation_maps(p, d, q)
    for k in range(K):
        s = int(b[k] * j0)
        want = np.full((H, W), 2, np.uint8)
        for u in range(W):
            if 0 <= u + s < W:
                want[:, u] = (q[k, :, u + s] >= 0.5)
        assert np.array_equal(lab[k], want), k


def test_segmentation_nearest_surface_wins_and_rounds_half_up():
    K, H, W, D = 2, 1, 12, 4
    p = _params(K, H, W, [0.0, 1.0], D, 100.0, ref=0)
    d = np.zeros((H, W), np.int32)
    d[0, 5], d[0, 4] = 2, 1             # both land on view-1 pixel 3: the larger disparity is seen
    q = np.zeros((K, H, W))
    q[1, 0, 5] = 1.0
    lab = O.segmentation_maps(p, d, q)
    assert lab[1, 0, 3] == 1
    q[1, 0, 5], q[1, 0, 4] = 0.0, 1.0
    assert O.segmentation_maps(p, d, q)[1, 0, 3] == 0
    # half a pixel: u = x - 0.5 is taken to pixel x
    p = _params(K, H, W, [0.0, 0.5], D, 100.0, ref=0)
    d = np.ones((H, W), np.int32)
    q = np.zeros((K, H, W))
    q[1, 0, 7] = 0.75
    lab = O.segmentation_maps(p, d, q)
    assert lab[1, 0, 7] == 1 and lab[1, 0, 6] == 0 and (lab[1, 0] != 2).all()


# ---------------------------------------------------------------- disparity prior construction

def _plane_views(K, H, W, b, d0, rng, period=None):
    """Views of one fronto-parallel textured plane at integer disparity d0:
    view k pixel x shows texture column x + b_k d0 (same row)."""
    pad = int(max(abs(v) for v in b) * d0) + 2
    if period:
        base = rng.integers(0, 256, size=(H, period, 3))
        tex = np.tile(base, (1, (W + 2 * pad) // period + 2, 1))[:, :W + 2 * pad]
    else:
        tex = rng.integers(0, 256, size=(H, W + 2 * pad, 3))
    views = np.zeros((K, H, W, 3), np.uint8)
    for k in range(K):
        s = int(b[k] * d0)
        views[k] = tex[:, pad + s:pad + s + W]
    return views


def test_support_points_recover_a_plane():
    rng = np.random.default_rng(60)
    K, H, W, D, d0 = 5, 40, 80, 16, 5
    b = [-2.0, -1.0, 0.0, 1.0, 2.0]
    views = _plane_views(K, H, W, b, d0, rng)
    p = _params(K, H, W, b, D, 100.0, ref=2)
    pts = O.support_points(p, O.make_support_params(), views, np.ones((K, H, W), np.float32))
    xs, ys = np.arange(2, W, 5), np.arange(2, H, 5)
    assert len(pts) == len(xs) * len(ys)                 # every grid point, all from the reference
    assert np.all(pts[:, 2] == d0) and np.all(pts[:, 3] == 2)
    assert np.array_equal(pts[:, :2], np.array([(x, y) for y in ys for x in xs]))


def test_support_points_fill_the_occluded_part_from_other_views():
    """A dynamic square in the reference only: no reference point inside it,
    points transferred from the other views at the plane's level instead."""
    rng = np.random.default_rng(61)
    K, H, W, D, d0 = 5, 40, 90, 16, 4
    b = [-2.0, -1.0, 0.0, 1.0, 2.0]
    views = _plane_views(K, H, W, b, d0, rng)
    views[2, 10:30, 30:60] = rng.integers(0, 256, size=(20, 30, 3))
    S_P = np.ones((K, H, W), np.float32)
    S_P[2, 10:30, 30:60] = 0.0
    p = _params(K, H, W, b, D, 100.0, ref=2)
    pts = O.support_points(p, O.make_support_params(), views, S_P)
    inside = (pts[:, 1] >= 10) & (pts[:, 1] < 30) & (pts[:, 0] >= 30) & (pts[:, 0] < 60)
    assert inside.sum() > 20
    assert np.all(pts[inside, 3] != 2) and np.all(pts[~inside, 3] == 2)
    assert np.all(pts[:, 2] == d0)
    # a transferred point came from a grid point of its view: x_a = u - b_a d0
    xa = pts[inside, 0] - np.array(b)[pts[inside, 3]].astype(int) * d0
    assert np.all((xa - 2) % 5 == 0)
    # one point per reference pixel, sorted by (y, u)
    key = pts[:, 1].astype(np.int64) * W + pts[:, 0]
    assert np.all(np.diff(key) > 0)


def test_support_points_need_texture_uniqueness_and_neighbours():
    rng = np.random.default_rng(62)
    K, H, W, D = 3, 30, 60, 12
    b = [-1.0, 0.0, 1.0]
    p = _params(K, H, W, b, D, 100.0, ref=1)
    ones = np.ones((K, H, W), np.float32)
    flat = np.full((K, H, W, 3), 128, np.uint8)
    assert len(O.support_points(p, O.make_support_params(), flat, ones)) == 0          # no texture
    periodic = _plane_views(K, H, W, b, 3, rng, period=4)                               # ambiguous along x
    assert len(O.support_points(p, O.make_support_params(), periodic, ones)) == 0
    plane = _plane_views(K, H, W, b, 3, rng)
    assert len(O.support_points(p, O.make_support_params(), plane, ones)) > 0
    lonely = O.make_support_params(incon_min=10 ** 6)                                   # nobody agrees
    assert len(O.support_points(p, lonely, plane, ones)) == 0
    dynamic = ones.copy()
    dynamic[1] = 0.0                                                                    # reference all dynamic,
    dynamic[0] = 0.0                                                                    # and the only other view
    assert len(O.support_points(p, O.make_support_params(), plane, dynamic)) == 0       # with a neighbour too


def test_raster_prior_is_scipy_linear_interpolation():
    from scipy.interpolate import LinearNDInterpolator
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(63)
    H, W, D = 50, 70, 40
    n = 60
    u = rng.choice(W, n, replace=True)
    y = rng.choice(H, n, replace=True)
    uy = np.unique(np.stack([u, y], 1), axis=0)
    lev = rng.integers(0, D, len(uy))
    pts = np.zeros((len(uy), 4), np.int32)
    pts[:, 0], pts[:, 1], pts[:, 2] = uy[:, 0], uy[:, 1], lev
    p = _params(3, H, W, [-1, 0, 1], D, 100.0, ref=1, d_min=-2.0, d_step=0.5)
    tri = Delaunay(pts[:, :2].astype(float))
    mu = O.raster_prior(p, pts, tri.simplices)
    gy, gx = np.mgrid[0:H, 0:W]
    dval = -2.0 + 0.5 * pts[:, 2]
    lin = LinearNDInterpolator(tri, dval)(gx, gy)
    inside = ~np.isnan(lin)
    np.testing.assert_allclose(mu[inside], lin[inside], rtol=0, atol=1e-5)
    d2 = (gx[..., None] - pts[:, 0]) ** 2 + (gy[..., None] - pts[:, 1]) ** 2
    near = dval[np.argmin(d2, axis=-1)]
    assert np.array_equal(mu[~inside], near[~inside].astype(np.float32))


def test_support_points_rules_in_detail():
    rng = np.random.default_rng(64)
    K, H, W, D, d0 = 3, 30, 70, 12, 3
    b = [-1.0, 0.0, 1.0]
    p = _params(K, H, W, b, D, 100.0, ref=1)
    ones = np.ones((K, H, W), np.float32)
    plane = _plane_views(K, H, W, b, d0, rng)
    # texture below the threshold: unique matches, but no point
    faint = (plane // 64 + 126).astype(np.uint8)
    sp = O.make_support_params(texture_min=10 ** 6)
    assert len(O.support_points(p, O.make_support_params(texture_min=0), faint, ones)) > 0
    assert len(O.support_points(p, sp, faint, ones)) == 0
    # a dynamic grid point is dropped even when the rest of its window is static
    holes = ones.copy()
    holes[1, 2::5, 2::5] = 0.0
    assert len(O.support_points(p, O.make_support_params(), plane, holes)) == 0
    # smooth noisy texture: the neighbouring levels of the best one are not
    # its competitors (with them, most of these points would be rejected)
    from scipy.ndimage import gaussian_filter
    r2 = np.random.default_rng(65)
    smooth = gaussian_filter(r2.uniform(0, 255, size=(H, W + 20, 3)), sigma=(0, 4, 0))
    views = np.zeros((K, H, W, 3), np.uint8)
    for k in range(K):
        s = int(b[k] * d0)
        views[k] = np.clip(smooth[:, 10 + s:10 + s + W] + r2.normal(0, 5.0, (H, W, 3)), 0, 255).astype(np.uint8)
    pts = O.support_points(p, O.make_support_params(texture_min=0, incon_min=0), views, ones)
    assert len(pts) >= 45 and np.median(pts[:, 2]) == d0


def test_prior_corners_take_the_nearest_level():
    p = _params(3, 20, 30, [-1, 0, 1], 10, 100.0, ref=1)
    pts = np.array([[5, 5, 3, 1], [20, 10, 7, 0]], np.int32)
    out = O.prior_corners(p, pts)
    assert out.tolist()[2:] == [[0, 0, 3, -1], [29, 0, 7, -1], [0, 19, 3, -1], [29, 19, 7, -1]]
    pts = np.array([[0, 0, 4, 1], [20, 10, 7, 0]], np.int32)        # a point on a corner already
    assert len(O.prior_corners(p, pts)) == 5
    assert len(O.prior_corners(p, np.zeros((0, 4), np.int32))) == 0


# ---------------------------------------------------------------- rules at their exact boundaries

@pytest.mark.parametrize("d_min,d_step", [(0.0, 1.0), (-3.0, 0.5), (1.25, 0.75)])
def test_nearest_level_half_way_takes_the_lower_level(d_min, d_step):
    """A pixel that is not swept (dynamic-only, static reference ray) takes
    the level nearest mu_T; exactly half-way between two levels the lower one
    wins, as for the arg min's ties.  Checked against numpy's argmin (first
    index of the smallest distance) with mu_T on and next to half-way points,
    and beyond both ends of the level range."""
    K, H, W, D = 3, 4, 24, 10
    b = [-1.0, 0.0, 1.0]
    rng = np.random.default_rng(70)
    levels = d_min + d_step * np.arange(D, dtype=np.float64)
    half = (levels[:-1] + levels[1:]) / 2.0
    mu = np.concatenate([half, half + d_step / 8, half - d_step / 8, levels,
                         [levels[0] - 5 * d_step, levels[-1] + 5 * d_step, levels[0] - d_step / 2,
                          levels[-1] + d_step / 2]])
    assert np.all(mu.astype(np.float32) == mu)                 # every value exact in float32
    mu = np.resize(mu, H * W).astype(np.float32).reshape(H, W)
    views = rng.integers(0, 256, size=(K, H, W, 3), dtype=np.uint8)
    S_P = np.ones((K, H, W), np.float32)                       # every reference ray static: none swept
    p = _params(K, H, W, b, D, 400.0, ref=1, d_min=d_min, d_step=d_step, dyn_only=True)
    r = O.reconstruct(p, views, S_P, mu, 1)
    dist = np.abs(levels[None, None, :] - mu[..., None].astype(np.float64))
    assert np.array_equal(r["d_idx"], np.argmin(dist, axis=-1))
    n_half = int(np.isin(mu.astype(np.float64), half).sum())
    assert n_half >= len(half)


def test_empty_search_window_takes_the_lower_nearest_level():
    """A search window holding no level falls back to the level nearest
    mu_T, the lower one when mu_T is half-way (numpy's argmin)."""
    K, H, W, D = 3, 2, 16, 8
    b = [-1.0, 0.0, 1.0]
    rng = np.random.default_rng(71)
    views = rng.integers(0, 256, size=(K, H, W, 3), dtype=np.uint8)
    S_P = np.full((K, H, W), 0.9, np.float32)
    mu = np.resize(np.array([0.5, 1.5, 2.5, 3.5, 4.5, 5.5, 6.5, 3.25], np.float32), (H, W)).astype(np.float32)
    # levels 0, 1, ..., 7 with a window of 0.25: no level within it at a half-way mu
    p = _params(K, H, W, b, D, 400.0, ref=1, window=0.25)
    r = O.reconstruct(p, views, S_P, mu, 1)
    levels = np.arange(D, dtype=np.float64)
    want = np.argmin(np.abs(levels[None, None, :] - mu[..., None].astype(np.float64)), axis=-1)
    assert np.array_equal(r["d_idx"], want)


def test_support_point_window_with_exactly_static_min_static_pixels_is_kept():
    """A grid point is a support point when it and at least static_min
    pixels of its window are static: exactly static_min is enough, one fewer
    is not (the count is brute-forced here)."""
    rng = np.random.default_rng(72)
    K, H, W, D, d0 = 3, 30, 60, 12, 3
    b = [-1.0, 0.0, 1.0]
    plane = _plane_views(K, H, W, b, d0, rng)
    p = _params(K, H, W, b, D, 100.0, ref=1)
    sp = O.make_support_params()
    x0, y0 = 27, 12                                        # a grid point (2 + 5i)
    win = [(y0 + dy, x0 + dx) for dy in range(-2, 3) for dx in range(-2, 3) if (dy, dx) != (0, 0)]
    for n_dyn, kept in [(25 - sp.static_min, True), (26 - sp.static_min, False)]:
        S_P = np.ones((K, H, W), np.float32)
        for (yy, xx) in win[:n_dyn]:
            S_P[1, yy, xx] = 0.0
        n_static = int((S_P[1, y0 - 2:y0 + 3, x0 - 2:x0 + 3] >= np.float32(0.7)).sum())
        assert n_static == 25 - n_dyn
        pts = O.support_points(p, sp, plane, S_P)
        ref_pt = (pts[:, 0] == x0) & (pts[:, 1] == y0) & (pts[:, 3] == 1)
        assert ref_pt.any() == kept, (n_static, kept)


def test_consistency_filter_is_the_brute_force_count():
    """The consistency filter keeps a point with at least incon_min others
    within incon_radius pixels (Chebyshev) and incon_levels levels, bounds
    included: checked by brute force over the unfiltered points of a scene
    whose two planes lie exactly incon_levels apart."""
    rng = np.random.default_rng(73)
    K, H, W, D = 3, 40, 90, 16
    b = [-1.0, 0.0, 1.0]
    pad = 12
    tex = rng.integers(0, 256, size=(H, W + 2 * pad, 3))
    views = np.zeros((K, H, W, 3), np.uint8)
    for k in range(K):
        for x in range(W):
            d = 4 if x < W // 2 else 6                      # two planes, levels 4 and 6
            views[k, :, x] = tex[:, pad + x + int(b[k]) * d]
    ones = np.ones((K, H, W), np.float32)
    p = _params(K, H, W, b, D, 100.0, ref=1)
    raw = O.support_points(p, O.make_support_params(incon_min=0), views, ones)
    levels = set(raw[:, 2].tolist())
    assert {4, 6} <= levels
    for incon_levels, incon_min in [(2, 8), (2, 12), (1, 8), (3, 12)]:
        sp = O.make_support_params(incon_levels=incon_levels, incon_min=incon_min)
        got = O.support_points(p, sp, views, ones)
        du = np.abs(raw[:, None, 0] - raw[None, :, 0])
        dy = np.abs(raw[:, None, 1] - raw[None, :, 1])
        dl = np.abs(raw[:, None, 2] - raw[None, :, 2])
        near = (du <= 10) & (dy <= 10) & (dl <= incon_levels)
        np.fill_diagonal(near, False)
        want = raw[near.sum(axis=1) >= incon_min]
        assert np.array_equal(got, want), (incon_levels, incon_min)
    # the bound matters on this scene: pairs exactly two levels apart decide some points
    a = O.support_points(p, O.make_support_params(incon_levels=2, incon_min=12), views, ones)
    c = O.support_points(p, O.make_support_params(incon_levels=1, incon_min=12), views, ones)
    assert len(a) > len(c)


def test_transferred_points_landing_on_one_pixel_keep_the_lowest_view():
    """With the plane at a multiple of the grid step, the grid points of
    every non-reference view land on the same reference pixels: one point per
    pixel is kept, from the lowest view (view 0 sees the whole occluded part
    here)."""
    rng = np.random.default_rng(74)
    K, H, W, D, d0 = 5, 40, 100, 16, 5
    b = [-2.0, -1.0, 0.0, 1.0, 2.0]
    views = _plane_views(K, H, W, b, d0, rng)
    views[2, 10:30, 40:70] = rng.integers(0, 256, size=(20, 30, 3))
    S_P = np.ones((K, H, W), np.float32)
    S_P[2, 10:30, 40:70] = 0.0
    p = _params(K, H, W, b, D, 100.0, ref=2)
    pts = O.support_points(p, O.make_support_params(), views, S_P)
    moved = pts[:, 3] != 2
    assert moved.sum() > 20
    key = pts[:, 1].astype(np.int64) * W + pts[:, 0]
    assert len(np.unique(key)) == len(key)                  # one point per reference pixel
    assert np.all(pts[moved, 3] == 0)                       # the lowest view wins every collision
    # every view's grid point would have landed on these pixels
    for a in (1, 3, 4):
        xa = pts[moved, 0] - int(b[a]) * d0
        assert np.all((xa - 2) % 5 == 0)


def test_match_cost_tie_takes_the_lowest_level():
    """The two sides of the reference see the plane at adjacent levels j and
    j + 1 (view 0 at j, view 2 at j + 1), so the side-robust cost is exactly
    0 at both: the lower level is the match."""
    rng = np.random.default_rng(75)
    K, H, W, D, j = 3, 30, 80, 12, 4
    b = [-1.0, 0.0, 1.0]
    pad = 20
    tex = rng.integers(0, 256, size=(H, W + 2 * pad, 3))
    views = np.zeros((K, H, W, 3), np.uint8)
    views[0] = tex[:, pad - j:pad - j + W]                  # x + b_0 j
    views[1] = tex[:, pad:pad + W]
    views[2] = tex[:, pad + (j + 1):pad + (j + 1) + W]      # x + b_2 (j + 1)
    ones = np.ones((K, H, W), np.float32)
    p = _params(K, H, W, b, D, 100.0, ref=1)
    pts = O.support_points(p, O.make_support_params(), views, ones)
    inner = (pts[:, 0] >= 2 + 2 + j + 1) & (pts[:, 0] < W - 2 - 2 - j - 1)
    assert inner.sum() > 20
    assert np.all(pts[inner, 2] == j)


def test_prior_corner_takes_the_euclidean_nearest_point():
    """A corner takes the level of its nearest point in Euclidean distance:
    here the nearest in L1 (and in Chebyshev) is another point."""
    p = _params(3, 20, 30, [-1, 0, 1], 10, 100.0, ref=1)
    pts = np.array([[6, 0, 2, 1], [4, 4, 7, 1], [25, 15, 5, 1]], np.int32)
    out = O.prior_corners(p, pts)
    corner = out[(out[:, 0] == 0) & (out[:, 1] == 0)]
    d2 = (pts[:, 0] - 0.0) ** 2 + (pts[:, 1] - 0.0) ** 2
    l1 = np.abs(pts[:, 0]) + np.abs(pts[:, 1])
    assert np.argmin(d2) != np.argmin(l1)
    assert corner[0, 2] == pts[np.argmin(d2), 2] == 7
