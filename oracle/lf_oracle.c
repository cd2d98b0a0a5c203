/*
 * FP64 CPU oracle of the EM static-background reconstruction with a rectified
 * linear camera array (Kaveti, Katt and Singh, "Removing Dynamic Objects for
 * Static Scene Reconstruction using Light Fields", 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow and obviously correct
 * reference the GPU library is checked against.  It shares no code, header,
 * table or helper with the GPU library, and only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  Every value is a double;
 * every pixel is processed on its own, in the order the paper gives the
 * steps (Sec. III-F: each pixel is processed independently).
 *
 * Readings of the paper this file follows (each is listed with its reason in
 * the design notes of the repository):
 *   - descriptor f = (Gx, Gy) * 2^-12 of the 3x3 Sobel responses of
 *     L = R+G+B, replicated border (Sec. III-C, pixel likelihood);
 *   - view k is sampled at u = x - b_k * d on the same row, by linear
 *     interpolation along x with indices clamped to the image (Eq. 1 for a
 *     rectified linear array; non-integral shifts, Sec. III-F);
 *   - the variance of the pixel likelihood is weighted by the per-view static
 *     posterior q_k and normalised by K, i.e. beta' = beta / K multiplies
 *     C = sum_k q_k |f_k - m|^2 with m the q-weighted mean (Sec. III-C);
 *   - M-step energy E(d) = beta' C + ln(1+gamma) - ln(gamma + exp(-(d-mu)^2
 *     / (2 sigma^2))) minimised over the D levels, lowest level on ties
 *     (Sec. III-C, E(d); Eq. 6);
 *   - E-step: q_k = P(S_k = 1) from the pixel likelihood and the prior
 *     rho_k, the segmentation prior S_P of view k sampled at the ray's
 *     footprint x - b_k mu_T (Sec. III-D, Eq. 7); static likelihood
 *     exp(lambda - beta' e_k), dynamic likelihood 1 ("the dynamic pixels
 *     don't contribute", Sec. III-C); hard mode takes the arg max;
 *   - first iteration weights: q0_k = [rho_k >= tau], tau = 0.7 (Sec. III-F),
 *     M-step first (Sec. III-B);
 *   - objective L = ln prior(d) + sum_k logaddexp(a1_k, a0_k) (soft) or
 *     sum_k max(a1_k, a0_k) (hard), the quantity EM never decreases;
 *   - refocus with the views whose posterior is >= 0.5 (Eq. 2), keeping the
 *     reference colour where no view is static (Sec. IV-B);
 *   - enumeration modes (2, 3): the E-step as the paper states it, over all
 *     2^K labelings S of the rays (Sec. III-C, last sentence; Sec. III-D),
 *     with the variance of the static descriptors normalised by the number
 *     of static views (Sec. III-C, Var) and no constant between the static
 *     and dynamic likelihoods: log weight of S is
 *       sum_k ln P(S_k | rho_k) - beta Var_S,  Var_S = 0 for fewer than two
 *     static views.  Mode 2 returns the marginals P(S_k = 1), mode 3 the
 *     labeling of largest weight (ties: the largest mask, bit k = view k).
 *     The M-step is unchanged (weights q, beta' = beta / K).
 *   - work-avoiding variants (Sec. III-C, the prior "reduces the search
 *     space"; Sec. III-F / IV, refocusing only the dynamic pixels): with
 *     window > 0 the M-step takes the arg min over the levels within
 *     `window` of mu_T only (the level nearest mu_T when there is none);
 *     with dyn_only a pixel whose reference ray is static by the prior
 *     threshold (rho_ref >= tau) is not reconstructed: it keeps its weights,
 *     takes the level nearest mu_T, adds nothing to the objective and shows
 *     its reference colour (not a hole).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LFO_MAX_VIEWS 16

typedef struct {
    int32_t K, H, W, ref;
    double baselines[LFO_MAX_VIEWS];
    double d_min, d_step;
    int32_t D;
    double beta, lambda, gamma, sigma, tau;
    int32_t storage; /* 0: inputs used as given, 1: rounded to binary16, 2: rounded to bfloat16 */
    int32_t mode;    /* 0: soft posterior, 1: hard assignment, 2 / 3: enumeration over all
                        labelings with the paper's coupled variance, marginals / arg max */
    double window;   /* > 0: the M-step searches only the levels with |d - mu_T| <= window */
    int32_t dyn_only; /* 1: EM and refocus only where the reference ray is dynamic by the
                         prior threshold (rho_ref < tau); elsewhere the reference pixel */
} lfo_params;

/* ------------------------------------------------------------------------ */
/* Rounding to the storage formats (IEEE 754 binary16; bfloat16 = the upper  */
/* half of binary32), round to nearest, ties to even.                        */
/* ------------------------------------------------------------------------ */

static double round_to_format(double v, int precision_bits, int min_normal_exp)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    frexp(v, &e);                 /* |v| = m 2^e, 0.5 <= m < 1 */
    int lead = e - 1;             /* exponent of the leading bit */
    if (lead < min_normal_exp) lead = min_normal_exp;  /* subnormals: fixed quantum */
    double quantum = ldexp(1.0, lead - (precision_bits - 1));
    return nearbyint(v / quantum) * quantum;           /* default mode: ties to even */
}

double lfo_round_storage(double v, int32_t storage)
{
    if (storage == 1) return round_to_format(v, 11, -14);
    if (storage == 2) return round_to_format(v, 8, -126);
    return v;
}

/* ------------------------------------------------------------------------ */
/* Likelihood constant.  The static-view likelihood is read as a normalised  */
/* Gaussian in descriptor space, (beta'/pi)^(F/2) exp(-beta' |f - m|^2), and */
/* the dynamic one as uniform over the descriptor box [-R, R]^F with         */
/* R = 3060 * 2^-12 (largest Sobel response of L = R+G+B).  lambda is the    */
/* log ratio of their normalisers.                                           */
/* ------------------------------------------------------------------------ */

double lfo_derive_lambda(const lfo_params *p)
{
    const double F = 2.0;
    double bp = p->beta / p->K;
    double R = 3060.0 / 4096.0;
    const double pi = 3.14159265358979323846;
    return 0.5 * F * log(bp / pi) + F * log(2.0 * R);
}

/* ------------------------------------------------------------------------ */
/* Descriptors: 3x3 Sobel responses of the intensity sum (Sec. III-C).       */
/* f layout [K][H][W][2] = (Gx, Gy) * 2^-12.                                 */
/* ------------------------------------------------------------------------ */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static double intensity(const uint8_t *view, int H, int W, int x, int y)
{
    x = clampi(x, 0, W - 1);
    y = clampi(y, 0, H - 1);
    const uint8_t *px = view + ((size_t)y * W + x) * 3;
    return (double)px[0] + (double)px[1] + (double)px[2];
}

void lfo_descriptors(const lfo_params *p, const uint8_t *views, double *f, int32_t y0, int32_t y1)
{
    const int K = p->K, H = p->H, W = p->W;
    const double w[3] = {1.0, 2.0, 1.0};
    const double scale = 1.0 / 4096.0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < K; ++k)
        for (int y = y0; y < y1; ++y) {
            const uint8_t *view = views + (size_t)k * H * W * 3;
            for (int x = 0; x < W; ++x) {
                double gx = 0.0, gy = 0.0;
                for (int t = -1; t <= 1; ++t) {
                    gx += w[t + 1] * (intensity(view, H, W, x + 1, y + t) - intensity(view, H, W, x - 1, y + t));
                    gy += w[t + 1] * (intensity(view, H, W, x + t, y + 1) - intensity(view, H, W, x + t, y - 1));
                }
                double *o = f + (((size_t)k * H + y) * W + x) * 2;
                o[0] = lfo_round_storage(gx * scale, p->storage);
                o[1] = lfo_round_storage(gy * scale, p->storage);
            }
        }
}

/* Linear interpolation between a (t = 0) and b (t = 1), in the form that is
 * exact when a == b: a certain prior (S_P exactly 0 or 1 on both sides)
 * stays certain. */
static double lerp(double a, double b, double t) { return a + t * (b - a); }

/* Sample a row at real position u: linear interpolation, indices clamped.   */
static double sample_row(const double *row, int W, int stride, double u)
{
    double fl = floor(u);
    double t = u - fl;
    int i0 = clampi((int)fl, 0, W - 1);
    int i1 = clampi((int)fl + 1, 0, W - 1);
    return lerp(row[(size_t)i0 * stride], row[(size_t)i1 * stride], t);
}

/* ------------------------------------------------------------------------ */
/* Ray prior: S_P of view k at the footprint of the prior disparity, and the */
/* first-iteration weights by thresholding it (Sec. III-F).                  */
/* ------------------------------------------------------------------------ */

/* rho is the static prior of the ray into view k; omr = 1 - rho, the dynamic
 * prior, is interpolated from 1 - S_P directly so that it keeps its relative
 * accuracy when rho is close to 1 (the E-step takes its logarithm). */
void lfo_ray_prior(const lfo_params *p, const float *S_P, const float *mu_T, double *rho, double *omr,
                   double *q0, int32_t y0, int32_t y1)
{
    const int K = p->K, H = p->H, W = p->W;
#pragma omp parallel for schedule(static)
    for (int y = y0; y < y1; ++y) {
        double *row = (double *)malloc(sizeof(double) * (size_t)W);
        double *row1m = (double *)malloc(sizeof(double) * (size_t)W);
        for (int k = 0; k < K; ++k) {
            const float *sp = S_P + ((size_t)k * H + y) * W;
            for (int x = 0; x < W; ++x) {
                row[x] = lfo_round_storage((double)sp[x], p->storage);
                row1m[x] = 1.0 - row[x];
            }
            for (int x = 0; x < W; ++x) {
                double u = (double)x - p->baselines[k] * (double)mu_T[(size_t)y * W + x];
                double r = sample_row(row, W, 1, u);
                size_t i = ((size_t)k * H + y) * W + x;
                rho[i] = r;
                if (omr) omr[i] = sample_row(row1m, W, 1, u);
                if (q0) q0[i] = (r >= p->tau) ? 1.0 : 0.0;
            }
        }
        free(row);
        free(row1m);
    }
}

/* ------------------------------------------------------------------------ */
/* One EM iteration: M-step then E-step (Sec. III-B, III-C, III-D).          */
/* ------------------------------------------------------------------------ */

static double log_prior(const lfo_params *p, double d, double mu)
{
    double z = d - mu;
    return log(p->gamma + exp(-(z * z) / (2.0 * p->sigma * p->sigma)));
}

/* Level index nearest mu (clamped to the level range). */
static int nearest_level(const lfo_params *p, double mu)
{
    double j = nearbyint((mu - p->d_min) / p->d_step);
    if (j < 0.0) j = 0.0;
    if (j > p->D - 1) j = p->D - 1;
    return (int)j;
}

static double logaddexp(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log1p(exp(-fabs(a - b)));
}

/* Descriptors of all views for reference pixel (x, y) at disparity d. */
static void gather(const lfo_params *p, const double *f, int x, int y, double d, double out[][2])
{
    const int H = p->H, W = p->W;
    for (int k = 0; k < p->K; ++k) {
        const double *row = f + ((size_t)k * H + y) * W * 2;
        double u = (double)x - p->baselines[k] * d;
        out[k][0] = sample_row(row + 0, W, 2, u);
        out[k][1] = sample_row(row + 1, W, 2, u);
    }
}

/* q-weighted mean m and C = sum_k q_k |f_k - m|^2 (two passes).  With no
 * weight at all the mean is unweighted and C = 0. */
static double weighted_spread(int K, const double fk[][2], const double *q, double m[2])
{
    double Q = 0.0;
    for (int k = 0; k < K; ++k) Q += q[k];
    if (Q > 0.0) {
        m[0] = m[1] = 0.0;
        for (int k = 0; k < K; ++k) { m[0] += q[k] * fk[k][0]; m[1] += q[k] * fk[k][1]; }
        m[0] /= Q; m[1] /= Q;
        double C = 0.0;
        for (int k = 0; k < K; ++k) {
            double a = fk[k][0] - m[0], b = fk[k][1] - m[1];
            C += q[k] * (a * a + b * b);
        }
        return C;
    }
    m[0] = m[1] = 0.0;
    for (int k = 0; k < K; ++k) { m[0] += fk[k][0]; m[1] += fk[k][1]; }
    m[0] /= K; m[1] /= K;
    return 0.0;
}

/* Enumeration E-step (modes 2, 3) of one pixel at the chosen level: fk are
 * the descriptors there, lr1 / lr0 the logs of rho_k and 1 - rho_k.  Writes
 * q and returns the log of the summed weights (mode 2) or the largest log
 * weight (mode 3). */
static double enumerate_labelings(const lfo_params *p, const double fk[][2], const double *lr1,
                                  const double *lr0, double *q)
{
    const int K = p->K;
    const int n_masks = 1 << K;
    double best = -INFINITY, top = -INFINITY;
    int best_mask = 0;
    /* first pass: the largest log weight (scales the sums of the second) */
    for (int pass = 0; pass < 2; ++pass) {
        double Z = 0.0, acc[LFO_MAX_VIEWS] = {0};
        for (int mask = 0; mask < n_masks; ++mask) {
            double lw = 0.0;
            int n = 0;
            for (int k = 0; k < K; ++k) {
                if (mask >> k & 1) { lw += lr1[k]; ++n; }
                else lw += lr0[k];
            }
            double var = 0.0;
            if (n >= 2) {
                double m0 = 0.0, m1 = 0.0;
                for (int k = 0; k < K; ++k)
                    if (mask >> k & 1) { m0 += fk[k][0]; m1 += fk[k][1]; }
                m0 /= n;
                m1 /= n;
                for (int k = 0; k < K; ++k)
                    if (mask >> k & 1) {
                        double a = fk[k][0] - m0, b = fk[k][1] - m1;
                        var += a * a + b * b;
                    }
                var /= n;
            }
            lw -= p->beta * var;
            if (pass == 0) {
                if (lw >= best) { best = lw; best_mask = mask; }
            } else if (lw > -INFINITY) {
                double w = exp(lw - top);
                Z += w;
                for (int k = 0; k < K; ++k)
                    if (mask >> k & 1) acc[k] += w;
            }
        }
        if (pass == 0) {
            if (p->mode == 3) {
                for (int k = 0; k < K; ++k) q[k] = (best_mask >> k & 1) ? 1.0 : 0.0;
                return best;
            }
            top = best;
        } else {
            for (int k = 0; k < K; ++k) q[k] = acc[k] / Z;
            return top + log(Z);
        }
    }
    return 0.0;
}

void lfo_em_iteration(const lfo_params *p, double lambda, const double *f, const double *rho,
                      const double *omr, const float *mu_T, const double *q_in, double *q_out, int32_t *d_idx,
                      double *L_pix, double *E1, double *E2, int32_t y0, int32_t y1)
{
    const int K = p->K, H = p->H, W = p->W, D = p->D;
    const double bp = p->beta / K;
    const double c0 = log(1.0 + p->gamma);
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = y0; y < y1; ++y) {
        double fk[LFO_MAX_VIEWS][2], q[LFO_MAX_VIEWS], m[2];
        for (int x = 0; x < W; ++x) {
            const size_t pix = (size_t)y * W + x;
            const double mu = (double)mu_T[pix];
            for (int k = 0; k < K; ++k) q[k] = q_in[(size_t)k * H * W + pix];

            if (p->dyn_only && !(rho[(size_t)p->ref * H * W + pix] < p->tau)) {
                /* static reference ray: not reconstructed */
                for (int k = 0; k < K; ++k) q_out[(size_t)k * H * W + pix] = q[k];
                d_idx[pix] = nearest_level(p, mu);
                if (L_pix) L_pix[pix] = 0.0;
                if (E1) E1[pix] = -INFINITY;
                if (E2) E2[pix] = INFINITY;
                continue;
            }

            /* M-step: exhaustive search over the disparity levels (those
             * within the window around mu_T when it is set). */
            int best = 0, searched = 0;
            double e_best = INFINITY, e_second = INFINITY;
            for (int j = 0; j <= D; ++j) {
                int jj = j;
                if (j == D) {            /* empty window: the level nearest mu_T */
                    if (searched) break;
                    jj = nearest_level(p, mu);
                }
                double d = p->d_min + jj * p->d_step;
                if (j < D && p->window > 0.0 && !(fabs(d - mu) <= p->window)) continue;
                ++searched;
                gather(p, f, x, y, d, fk);
                double C = weighted_spread(K, fk, q, m);
                double E = bp * C + c0 - log_prior(p, d, mu);
                if (E < e_best) { e_second = e_best; e_best = E; best = jj; }
                else if (E < e_second) e_second = E;
            }

            /* E-step at the new disparity. */
            double d = p->d_min + best * p->d_step;
            gather(p, f, x, y, d, fk);
            weighted_spread(K, fk, q, m);
            double L = log_prior(p, d, mu);
            if (p->mode >= 2) {
                double lr1[LFO_MAX_VIEWS], lr0[LFO_MAX_VIEWS], qk[LFO_MAX_VIEWS];
                for (int k = 0; k < K; ++k) {
                    double r = rho[(size_t)k * H * W + pix];
                    double r1 = omr ? omr[(size_t)k * H * W + pix] : 1.0 - r;
                    lr1[k] = r > 0.0 ? log(r) : -INFINITY;
                    lr0[k] = r1 > 0.0 ? log(r1) : -INFINITY;
                }
                L += enumerate_labelings(p, fk, lr1, lr0, qk);
                for (int k = 0; k < K; ++k) q_out[(size_t)k * H * W + pix] = qk[k];
            }
            for (int k = 0; k < K && p->mode < 2; ++k) {
                double a = fk[k][0] - m[0], b = fk[k][1] - m[1];
                double e = a * a + b * b;
                double r = rho[(size_t)k * H * W + pix];
                double r1 = omr ? omr[(size_t)k * H * W + pix] : 1.0 - r;
                double a1 = (r > 0.0 ? log(r) : -INFINITY) + lambda - bp * e;
                double a0 = (r1 > 0.0 ? log(r1) : -INFINITY);
                double qk;
                if (p->mode == 1) {
                    qk = (a1 >= a0) ? 1.0 : 0.0;
                    L += (a1 >= a0) ? a1 : a0;
                } else {
                    qk = 1.0 / (1.0 + exp(a0 - a1));
                    L += logaddexp(a1, a0);
                }
                q_out[(size_t)k * H * W + pix] = qk;
            }
            d_idx[pix] = best;
            if (L_pix) L_pix[pix] = L;
            if (E1) E1[pix] = e_best;
            if (E2) E2[pix] = e_second;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Refocus with the static rays only (Eq. 2).  rgb in [0,1], [H][W][3].      */
/* ------------------------------------------------------------------------ */

void lfo_refocus(const lfo_params *p, const uint8_t *views, const int32_t *d_idx, const double *q,
                 const double *rho, double *rgb, uint8_t *hole, int32_t y0, int32_t y1)
{
    const int K = p->K, H = p->H, W = p->W;
#pragma omp parallel for schedule(static)
    for (int y = y0; y < y1; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t pix = (size_t)y * W + x;
            if (p->dyn_only && rho && !(rho[(size_t)p->ref * H * W + pix] < p->tau)) {
                /* static reference ray: the reference pixel is the background */
                const uint8_t *c_ref = views + (((size_t)p->ref * H + y) * W + x) * 3;
                for (int c = 0; c < 3; ++c) rgb[pix * 3 + c] = (double)c_ref[c] / 255.0;
                if (hole) hole[pix] = 0;
                continue;
            }
            double d = p->d_min + d_idx[pix] * p->d_step;
            double acc[3] = {0.0, 0.0, 0.0};
            int n = 0;
            for (int k = 0; k < K; ++k) {
                if (!(q[(size_t)k * H * W + pix] >= 0.5)) continue;
                const uint8_t *vr = views + (((size_t)k * H + y) * W) * 3;
                double u = (double)x - p->baselines[k] * d;
                for (int c = 0; c < 3; ++c) {
                    double fl = floor(u), t = u - fl;
                    int i0 = clampi((int)fl, 0, W - 1), i1 = clampi((int)fl + 1, 0, W - 1);
                    acc[c] += lerp((double)vr[(size_t)i0 * 3 + c], (double)vr[(size_t)i1 * 3 + c], t);
                }
                ++n;
            }
            double *o = rgb + pix * 3;
            if (n > 0) {
                for (int c = 0; c < 3; ++c) o[c] = acc[c] / (255.0 * n);
                if (hole) hole[pix] = 0;
            } else {
                const uint8_t *c_ref = views + (((size_t)p->ref * H + y) * W + x) * 3;
                for (int c = 0; c < 3; ++c) o[c] = (double)c_ref[c] / 255.0;
                if (hole) hole[pix] = 1;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Whole reconstruction of rows [y0, y1): descriptors, ray prior, n_iters EM */
/* iterations and the refocus.  Scratch buffers are the caller's; they are   */
/* full-frame sized so row bands index like whole frames.  q_warm may be     */
/* NULL (threshold start).  The final weights end in q_a and the last        */
/* iteration's per-pixel objective in L_pix.  Returns the OpenMP threads.    */
/* ------------------------------------------------------------------------ */

int32_t lfo_reconstruct(const lfo_params *p, const uint8_t *views, const float *S_P, const float *mu_T,
                        const double *q_warm, int32_t n_iters, int32_t y0, int32_t y1,
                        double *f, double *rho, double *omr, double *q_a, double *q_b,
                        int32_t *d_idx, double *L_pix, double *L_sum, double *rgb, uint8_t *hole)
{
    const int K = p->K, H = p->H, W = p->W;
    double lambda = isnan(p->lambda) ? lfo_derive_lambda(p) : p->lambda;
    lfo_descriptors(p, views, f, y0, y1);
    lfo_ray_prior(p, S_P, mu_T, rho, omr, q_a, y0, y1);
    if (q_warm)
        for (int k = 0; k < K; ++k)
            memcpy(q_a + ((size_t)k * H + y0) * W, q_warm + ((size_t)k * H + y0) * W,
                   sizeof(double) * (size_t)(y1 - y0) * W);
    for (int t = 0; t < n_iters; ++t) {
        lfo_em_iteration(p, lambda, f, rho, omr, mu_T, q_a, q_b, d_idx, L_pix, NULL, NULL, y0, y1);
        if (L_sum) {
            double s = 0.0;
            for (int y = y0; y < y1; ++y)
                for (int x = 0; x < W; ++x) s += L_pix[(size_t)y * W + x];
            L_sum[t] = s;
        }
        double *tmp = q_a; q_a = q_b; q_b = tmp;
    }
    lfo_refocus(p, views, d_idx, q_a, rho, rgb, hole, y0, y1);
    /* leave the final weights in the caller's first buffer */
    if (n_iters % 2 == 1)
        for (int k = 0; k < K; ++k)
            memcpy(q_b + ((size_t)k * H + y0) * W, q_a + ((size_t)k * H + y0) * W,
                   sizeof(double) * (size_t)(y1 - y0) * W);
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int32_t lfo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* 3x3 per-channel median of the refocused image, replicated border: the     */
/* filter that removes the specular noise of the pixel-wise refocus          */
/* (Sec. III-E).  rgb and out are [H][W][3].                                 */
/* ------------------------------------------------------------------------ */

void lfo_median3(const lfo_params *p, const double *rgb, double *out, int32_t y0, int32_t y1)
{
    const int H = p->H, W = p->W;
#pragma omp parallel for schedule(static)
    for (int y = y0; y < y1; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < 3; ++c) {
                double v[9];
                int n = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int yy = clampi(y + dy, 0, H - 1), xx = clampi(x + dx, 0, W - 1);
                        double a = rgb[((size_t)yy * W + xx) * 3 + c];
                        int i = n++;
                        while (i > 0 && v[i - 1] > a) { v[i] = v[i - 1]; --i; }
                        v[i] = a;
                    }
                out[((size_t)y * W + x) * 3 + c] = v[4];
            }
}

/* ------------------------------------------------------------------------ */
/* Per-view segmentation maps in each view's own pixel grid (the updated     */
/* segmentation of Sec. III-D shown per view, as in the paper's figures).    */
/* The ray of reference pixel (x, y) at its level d lands in view k at       */
/* u = x - b_k d on row y, taken to the nearest pixel floor(u + 1/2).  Where */
/* several rays land on one pixel the one with the largest disparity (the    */
/* nearest surface) is seen; labels are 1 (static, q_k >= 1/2), 0 (dynamic)  */
/* and 2 (no reference ray lands there).  labels is uint8 [K][H][W].         */
/* ------------------------------------------------------------------------ */

void lfo_segmentation_maps(const lfo_params *p, const int32_t *d_idx, const double *q, uint8_t *labels,
                           int32_t y0, int32_t y1)
{
    const int K = p->K, H = p->H, W = p->W;
#pragma omp parallel for schedule(static)
    for (int y = y0; y < y1; ++y) {
        int *winner = (int *)malloc(sizeof(int) * (size_t)W);
        for (int k = 0; k < K; ++k) {
            for (int u = 0; u < W; ++u) winner[u] = -1;
            for (int x = 0; x < W; ++x) {
                const int j = d_idx[(size_t)y * W + x];
                const double u = (double)x - p->baselines[k] * (p->d_min + j * p->d_step);
                const double ur = floor(u + 0.5);
                if (ur < 0.0 || ur > W - 1) continue;
                const int iu = (int)ur;
                const int w = winner[iu];
                if (w < 0 || j > d_idx[(size_t)y * W + w]) winner[iu] = x;
            }
            for (int u = 0; u < W; ++u) {
                uint8_t *l = labels + ((size_t)k * H + y) * W + u;
                if (winner[u] < 0) *l = 2;
                else *l = q[((size_t)k * H + y) * W + winner[u]] >= 0.5 ? 1 : 0;
            }
        }
        free(winner);
    }
}
