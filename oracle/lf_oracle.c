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

/* Level index nearest mu (clamped to the level range).  A mu exactly
 * half-way between two levels takes the lower one, the same rule as the arg
 * min's ties.  The quotient is formed in double from the single-precision
 * mu, d_min and d_step, so a half-way point is seen exactly. */
static int nearest_level(const lfo_params *p, double mu)
{
    double j = ceil((mu - p->d_min) / p->d_step - 0.5);
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

/* ------------------------------------------------------------------------ */
/* Disparity prior construction (Sec. III-C, disparity prior): support       */
/* points matched along the epipolar line over the full disparity range,     */
/* those on dynamic objects dropped, support points of the other views       */
/* transferred into the reference where it is occluded by a dynamic object,  */
/* duplicates and inconsistent points removed; then the prior mu_T is the    */
/* piecewise-linear interpolation over a triangulation of the points.        */
/*                                                                            */
/* Readings (the paper follows ELAS and gives no numbers):                    */
/*  - matching uses the integer Sobel responses (Gx, Gy) of L = R+G+B and    */
/*    the sum of absolute differences over a (2r+1)^2 window, summed over    */
/*    the views matched against, borders replicated; integer geometry only   */
/*    (integer baselines and levels);                                         */
/*  - a candidate is kept when its window has texture (sum of |Gx| + |Gy|    */
/*    >= texture_min) and its best cost is unique: best * den < second *     */
/*    num, the second best taken over levels at least 2 away; ties of the    */
/*    best go to the lowest level;                                            */
/*  - the views on either side of the matched view are summed apart and the */
/*    smaller of the two sums is the cost (one side usually sees past an     */
/*    occluder); a view at the end of the array has one side;                */
/*  - reference pass: grid points of the reference matched against every     */
/*    other view, kept where the point and at least static_min pixels of its */
/*    window are static in the reference (S_P >= tau);                       */
/*  - transfer pass: grid points of each other view a matched against its    */
/*    non-reference neighbours a-1, a+1, static in view a as above, moved to */
/*    reference column u = x + b_a d and kept where the reference is         */
/*    dynamic there (S_P_ref < tau, the occluded part); of several points    */
/*    landing on one reference pixel the one of the lowest view (then the    */
/*    lowest x) is kept;                                                      */
/*  - consistency: a point is kept when at least incon_min other points lie  */
/*    within incon_radius pixels (Chebyshev) with levels within              */
/*    incon_levels;                                                           */
/*  - points are reported sorted by (y, u).                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t step, radius, texture_min, ratio_num, ratio_den;
    int32_t incon_radius, incon_levels, incon_min, static_min;
} lfo_support_params;

/* Integer Sobel responses of view k, [H][W][2]. */
static void sobel_int(const lfo_params *p, const uint8_t *views, int k, int32_t *g)
{
    const int H = p->H, W = p->W;
    const uint8_t *v = views + (size_t)k * H * W * 3;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int L[3][3];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) L[r][c] = (int)intensity(v, H, W, x + c - 1, y + r - 1);
            g[((size_t)y * W + x) * 2 + 0] = (L[0][2] - L[0][0]) + 2 * (L[1][2] - L[1][0]) + (L[2][2] - L[2][0]);
            g[((size_t)y * W + x) * 2 + 1] = (L[2][0] - L[0][0]) + 2 * (L[2][1] - L[0][1]) + (L[2][2] - L[0][2]);
        }
}

/* Whether the grid point (x, y) is static in view a by the prior threshold
 * (S_P >= tau) and at least static_min pixels of its matching window are. */
static int window_static(const lfo_params *p, const lfo_support_params *sp, const float *S_P, int a, int x, int y)
{
    const int H = p->H, W = p->W, r = sp->radius;
    const float tau = (float)p->tau;
    if (!(S_P[((size_t)a * H + y) * W + x] >= tau)) return 0;
    int n = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            n += S_P[((size_t)a * H + clampi(y + dy, 0, H - 1)) * W + clampi(x + dx, 0, W - 1)] >= tau;
    return n >= sp->static_min;
}

/* Level of the unique best match of grid point (x, y) of view a against the
 * views in vs (n_vs of them), or -1. */
static int match_point(const lfo_params *p, const lfo_support_params *sp, int32_t *const *G, int a, const int *vs,
                       int n_vs, int x, int y)
{
    const int H = p->H, W = p->W, D = p->D, r = sp->radius;
    long texture = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            const int32_t *ga = G[a] + ((size_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)) * 2;
            texture += labs((long)ga[0]) + labs((long)ga[1]);
        }
    if (texture < sp->texture_min) return -1;
    long *cost = (long *)malloc(sizeof(long) * (size_t)D);
    for (int j = 0; j < D; ++j) {
        const double d = p->d_min + j * p->d_step;
        /* the views on either side of view a are summed apart and the
         * smaller sum is the cost: one side usually sees past an occluder */
        long side[2] = {0, 0};
        int used[2] = {0, 0};
        for (int i = 0; i < n_vs; ++i) {
            const int v = vs[i];
            const int sd = p->baselines[v] > p->baselines[a];
            used[sd] = 1;
            const int shift = (int)lround((p->baselines[v] - p->baselines[a]) * d);
            for (int dy = -r; dy <= r; ++dy) {
                const int yy = clampi(y + dy, 0, H - 1);
                for (int dx = -r; dx <= r; ++dx) {
                    const int32_t *ga = G[a] + ((size_t)yy * W + clampi(x + dx, 0, W - 1)) * 2;
                    const int32_t *gv = G[v] + ((size_t)yy * W + clampi(x + dx - shift, 0, W - 1)) * 2;
                    side[sd] += labs((long)ga[0] - gv[0]) + labs((long)ga[1] - gv[1]);
                }
            }
        }
        cost[j] = (used[0] && used[1]) ? (side[0] < side[1] ? side[0] : side[1]) : side[0] + side[1];
    }
    int best = 0;
    for (int j = 1; j < D; ++j)
        if (cost[j] < cost[best]) best = j;
    long second = -1;
    for (int j = 0; j < D; ++j)
        if (abs(j - best) >= 2 && (second < 0 || cost[j] < second)) second = cost[j];
    const int ok = second >= 0 ? cost[best] * sp->ratio_den < second * sp->ratio_num : 1;
    free(cost);
    return ok ? best : -1;
}

static int cmp_points(const void *pa, const void *pb)
{
    const int32_t *a = (const int32_t *)pa, *b = (const int32_t *)pb;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;   /* y */
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;   /* u */
    return 0;
}

/* points: int32 [max_points][4] = (u, y, level, view).  Returns the number of
 * points kept (at most max_points are written), or -1 on a bad argument. */
int32_t lfo_support_points(const lfo_params *p, const lfo_support_params *sp, const uint8_t *views, const float *S_P,
                           int32_t *points, int32_t max_points)
{
    const int K = p->K, H = p->H, W = p->W, s = sp->step;
    if (s < 1 || sp->radius < 0) return -1;
    int32_t **G = (int32_t **)malloc(sizeof(int32_t *) * (size_t)K);
    for (int k = 0; k < K; ++k) {
        G[k] = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W * 2);
        sobel_int(p, views, k, G[k]);
    }
    const float tau = (float)p->tau;
    const int nx = (W - s / 2 + s - 1) / s, ny = (H - s / 2 + s - 1) / s;
    /* candidates: reference pass, then transfer pass view by view */
    size_t cap = (size_t)nx * ny * K + 1, n = 0;
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
    int32_t *level = (int32_t *)malloc(sizeof(int32_t) * (size_t)nx * ny);
    {
        int vs[LFO_MAX_VIEWS], n_vs = 0;
        for (int k = 0; k < K; ++k)
            if (k != p->ref) vs[n_vs++] = k;
#pragma omp parallel for schedule(dynamic, 1)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const int x = s / 2 + ix * s, y = s / 2 + iy * s;
                int j = -1;
                if (window_static(p, sp, S_P, p->ref, x, y)) j = match_point(p, sp, G, p->ref, vs, n_vs, x, y);
                level[(size_t)iy * nx + ix] = j;
            }
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const int j = level[(size_t)iy * nx + ix];
                if (j < 0) continue;
                int32_t *c = cand + 4 * n++;
                c[0] = s / 2 + ix * s; c[1] = s / 2 + iy * s; c[2] = j; c[3] = p->ref;
            }
    }
    const size_t n_ref = n;
    uint8_t *taken = (uint8_t *)calloc((size_t)H * W, 1);
    for (int a = 0; a < K; ++a) {
        if (a == p->ref) continue;
        int vs[2], n_vs = 0;
        if (a - 1 >= 0 && a - 1 != p->ref) vs[n_vs++] = a - 1;
        if (a + 1 < K && a + 1 != p->ref) vs[n_vs++] = a + 1;
        if (n_vs == 0) continue;
#pragma omp parallel for schedule(dynamic, 1)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const int x = s / 2 + ix * s, y = s / 2 + iy * s;
                int j = -1;
                if (window_static(p, sp, S_P, a, x, y)) j = match_point(p, sp, G, a, vs, n_vs, x, y);
                level[(size_t)iy * nx + ix] = j;
            }
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const int j = level[(size_t)iy * nx + ix];
                if (j < 0) continue;
                const int x = s / 2 + ix * s, y = s / 2 + iy * s;
                const int u = x + (int)lround(p->baselines[a] * (p->d_min + j * p->d_step));
                if (u < 0 || u >= W) continue;
                if (!(S_P[((size_t)p->ref * H + y) * W + u] < tau)) continue;
                if (taken[(size_t)y * W + u]) continue;
                taken[(size_t)y * W + u] = 1;
                int32_t *c = cand + 4 * n++;
                c[0] = u; c[1] = y; c[2] = j; c[3] = a;
            }
    }
    (void)n_ref;
    /* consistency with the neighbours */
    int32_t kept = 0;
    uint8_t *keep = (uint8_t *)calloc(n + 1, 1);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) {
        int cnt = 0;
        for (size_t m = 0; m < n; ++m) {
            if (m == i) continue;
            if (abs(cand[4 * m] - cand[4 * i]) <= sp->incon_radius &&
                abs(cand[4 * m + 1] - cand[4 * i + 1]) <= sp->incon_radius &&
                abs(cand[4 * m + 2] - cand[4 * i + 2]) <= sp->incon_levels)
                ++cnt;
        }
        keep[i] = cnt >= sp->incon_min;
    }
    int32_t *out = (int32_t *)malloc(sizeof(int32_t) * 4 * (n + 1));
    for (size_t i = 0; i < n; ++i)
        if (keep[i]) { memcpy(out + 4 * kept, cand + 4 * i, sizeof(int32_t) * 4); ++kept; }
    qsort(out, (size_t)kept, sizeof(int32_t) * 4, cmp_points);
    memcpy(points, out, sizeof(int32_t) * 4 * (size_t)(kept < max_points ? kept : max_points));
    free(out); free(keep); free(taken); free(level); free(cand);
    for (int k = 0; k < K; ++k) free(G[k]);
    free(G);
    return kept;
}

/* mu_T from support points and a triangulation of them: in a triangle the   */
/* disparity is the barycentric interpolation of its corners' levels (exact  */
/* integer areas; the first triangle containing the pixel, edges included);  */
/* outside every triangle, the disparity of the nearest point (lowest index  */
/* on ties); with no point at all, the middle of the level range.  points    */
/* int32 [n][4] as above, tris int32 [n_tri][3].                             */
void lfo_raster_prior(const lfo_params *p, const int32_t *points, int32_t n, const int32_t *tris, int32_t n_tri,
                      float *mu_T)
{
    const int H = p->H, W = p->W;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double mu = NAN;
            for (int t = 0; t < n_tri && isnan(mu); ++t) {
                const int32_t *a = points + 4 * tris[3 * t], *b = points + 4 * tris[3 * t + 1],
                              *c = points + 4 * tris[3 * t + 2];
                const long A = (long)(b[0] - a[0]) * (c[1] - a[1]) - (long)(b[1] - a[1]) * (c[0] - a[0]);
                if (A == 0) continue;
                const long wa = (long)(b[0] - x) * (c[1] - y) - (long)(b[1] - y) * (c[0] - x);
                const long wb = (long)(c[0] - x) * (a[1] - y) - (long)(c[1] - y) * (a[0] - x);
                const long wc = (long)(a[0] - x) * (b[1] - y) - (long)(a[1] - y) * (b[0] - x);
                const int inside = A > 0 ? (wa >= 0 && wb >= 0 && wc >= 0) : (wa <= 0 && wb <= 0 && wc <= 0);
                if (!inside) continue;
                const double da = p->d_min + a[2] * p->d_step, db = p->d_min + b[2] * p->d_step,
                             dc = p->d_min + c[2] * p->d_step;
                mu = ((double)wa * da + (double)wb * db + (double)wc * dc) / (double)A;
            }
            if (isnan(mu) && n == 0) mu = p->d_min + 0.5 * (p->D - 1) * p->d_step;   /* no point at all */
            if (isnan(mu)) {
                long best = -1;
                for (int i = 0; i < n; ++i) {
                    const long dx = points[4 * i] - x, dy = points[4 * i + 1] - y, d2 = dx * dx + dy * dy;
                    if (best < 0 || d2 < best) { best = d2; mu = p->d_min + points[4 * i + 2] * p->d_step; }
                }
            }
            mu_T[(size_t)y * W + x] = (float)mu;
        }
}

/* The four image corners as extra points (as ELAS does), each with the level
 * of the nearest support point (squared distance, lowest index on ties), so
 * that the triangulation covers the whole frame; a corner already holding a
 * point is not added.  points int32 [n + 4][4] (room for four more); view
 * = -1 marks a corner.  Returns the new count (n when n == 0). */
int32_t lfo_prior_corners(const lfo_params *p, int32_t *points, int32_t n)
{
    const int cx[4] = {0, p->W - 1, 0, p->W - 1}, cy[4] = {0, 0, p->H - 1, p->H - 1};
    int32_t m = n;
    if (n == 0) return 0;
    for (int c = 0; c < 4; ++c) {
        int dup = 0;
        for (int i = 0; i < m; ++i)
            if (points[4 * i] == cx[c] && points[4 * i + 1] == cy[c]) dup = 1;
        if (dup) continue;
        long best = -1;
        int lev = 0;
        for (int i = 0; i < n; ++i) {
            const long dx = points[4 * i] - cx[c], dy = points[4 * i + 1] - cy[c], d2 = dx * dx + dy * dy;
            if (best < 0 || d2 < best) { best = d2; lev = points[4 * i + 2]; }
        }
        int32_t *q = points + 4 * m++;
        q[0] = cx[c]; q[1] = cy[c]; q[2] = lev; q[3] = -1;
    }
    return m;
}
