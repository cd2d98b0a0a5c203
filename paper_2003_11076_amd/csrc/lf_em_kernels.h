// Device code of the EM static-background reconstruction for gfx950: the
// storage formats, footprint helpers and the fused EM kernel
//   lf_em_kernel   n EM iterations: M-step sweep over all disparity levels
//                  (Eq. 6, E(d)), E-step posterior (Eq. 7), per-pixel
//                  objective and its FP64 block sums
// The per-frame kernels before and after it are in lf_frame_kernels.h.
// Every pixel is processed independently (Sec. III-F).
//
// A rectified linear array shifts views along x only, so the EM kernel stages
// one row tile of every view plus its disparity halo in LDS once per launch
// and sweeps all levels and iterations from there; one lane owns one pixel.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

namespace lfem {

constexpr int kMaxViews = 16;
constexpr float kLn2 = 0.69314718055994530942f;

// ---------------------------------------------------------------------------
// Storage of one descriptor pair (Gx, Gy).
// ---------------------------------------------------------------------------
template <int ST> struct Pair;
template <> struct Pair<0> { using T = float2; };    // FP32
template <> struct Pair<1> { using T = __half2; };   // binary16
template <> struct Pair<2> { using T = uint32_t; };  // bfloat16: low half Gx, high half Gy

__device__ __forceinline__ float2 widen(float2 v) { return v; }
__device__ __forceinline__ float2 widen(__half2 v) { return __half22float2(v); }
__device__ __forceinline__ float2 widen(uint32_t v) {
    return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
}

// Round a float to bfloat16, to nearest with ties to even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <int ST> __device__ __forceinline__ typename Pair<ST>::T make_pair(float gx, float gy);
template <> __device__ __forceinline__ float2 make_pair<0>(float gx, float gy) { return make_float2(gx, gy); }
template <> __device__ __forceinline__ __half2 make_pair<1>(float gx, float gy) {
    return __halves2half2(__float2half_rn(gx), __float2half_rn(gy));
}
template <> __device__ __forceinline__ uint32_t make_pair<2>(float gx, float gy) {
    return bf16_bits_rne(gx) | (bf16_bits_rne(gy) << 16);
}

// A value as held in the given storage precision, widened back to float.
__device__ __forceinline__ float as_stored(float v, int st) {
    if (st == 1) return __half2float(__float2half_rn(v));
    if (st == 2) return __uint_as_float(bf16_bits_rne(v) << 16);
    return v;
}

// Linear interpolation written so that equal neighbours give that value
// exactly (a certain prior S_P in {0, 1} stays certain) and t = 0 gives a.
__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

// Footprint u = x - b * d split into floor(u) and frac(u) with the product
// b*d taken exactly (Dekker's two-product via fma), so the fractional part is
// accurate to a few units of 2^-24 whatever the size of x and b*d.
__device__ __forceinline__ void footprint(int x, float b, float d, int &i0, float &frac) {
    // no contraction here: fusing t - floor(t) into fma(b, d, -floor(t))
    // would fold the product's rounding error into s and count it twice
#pragma clang fp contract(off)
    float t = b * d;
    float err = fmaf(b, d, -t);      // b*d = t + err exactly
    float fl = floorf(t);
    float s = t - fl;                 // exact
    float r = -(s + err);             // u = (x - fl) + r, r in about (-1, 0]
    float fr = floorf(r);
    i0 = x - (int)fl + (int)fr;
    frac = r - fr;
}

// The same footprint with both t = frac(u) and 1 - t returned to full
// relative precision (each is formed from the exact product's pieces rather
// than as a difference of nearly equal numbers); used where a prior that is
// nearly 0 or nearly 1 must keep its relative accuracy.
__device__ __forceinline__ void footprint_precise(int x, float b, float d, int &i0, float &t, float &omt) {
#pragma clang fp contract(off)
    const float th = b * d;
    const float err = fmaf(b, d, -th);   // b*d = th + err exactly
    const float fl = floorf(th);
    const float s = th - fl;              // exact, in [0, 1)
    const float F = s + err;              // frac(b d), up to rounding; picks the case
    const int base = x - (int)fl;
    if (F <= 0.0f) {                      // u = base + (-s - err), 0 <= -s - err < 1
        i0 = base;
        t = (-s) - err;
        omt = 1.0f - t;
    } else if (F < 1.0f) {                // u = base - 1 + (1 - s - err)
        i0 = base - 1;
        t = (1.0f - s) - err;
        omt = s + err;
    } else {                              // s close to 1 and err > 0
        i0 = base - 2;
        omt = (s - 1.0f) + err;
        t = 1.0f - omt;
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Ray prior of one ray (Sec. III-B): S_P of the view (held in the storage
// precision) interpolated at the footprint x - b mu, and its complement
// interpolated from 1 - S_P; both from the nearer end of the interval so they
// keep their relative accuracy as they approach 0 (the E-step takes their
// logarithms).
__device__ __forceinline__ void ray_prior_value(const float *row, int W, int x, float b, float mu, int storage,
                                                float &rho, float &omr) {
    int i0;
    float t, omt;
    footprint_precise(x, b, mu, i0, t, omt);
    const float s0 = as_stored(row[clampi(i0, 0, W - 1)], storage);
    const float s1 = as_stored(row[clampi(i0 + 1, 0, W - 1)], storage);
    if (t <= 0.5f) {
        rho = fmaf(t, s1 - s0, s0);
        omr = fmaf(-t, s1 - s0, 1.0f - s0);
    } else {
        rho = fmaf(omt, s0 - s1, s1);
        omr = fmaf(-omt, s0 - s1, 1.0f - s1);
    }
}

// ---------------------------------------------------------------------------
// EM iterations.  grid (ceil(W/tile), H), block = tile threads, one pixel per
// lane.  Dynamic LDS: for every view, the tile's descriptor window plus its
// disparity halo, one record per position holding (Gx, Gy) at storage
// precision and the squared norm |f|^2 in FP32.
//
// Views are processed in "kernel order": kernel view 0 is the reference view
// (baseline 0), whose descriptor does not move with the level and is kept in
// registers; perm[k] maps kernel order to the [K][H][W] array index.
//
// The M-step sweep scores each level with the one-pass energy
//   E^ = beta' (S - |A|^2 / W) - P_j,  A = sum w_k f_k, S = sum w_k |f_k|^2,
// (3 FMAs per view) and re-evaluates a level exactly, with the two-pass
// weighted spread of the exhaustive sweep, whenever it could beat the best
// exact energy so far: E^ - M <= E_best, M = beta' margin_k S + margin_c a
// bound of |E^ - E| for this formula in FP32 (margin_k carries a factor 4
// of slack over the bound, which also covers the folded form evaluated).  The sweep is seeded with the
// previous iteration's level, so re-evaluations are rare, and the arg min and
// tie rule (lowest level) are exactly those of the exhaustive sweep.  The
// prior term is evaluated only inside a wave-uniform window |d - mu| <= T;
// outside it gamma + g rounds to gamma in FP32, so the constant used there is
// bit-identical to the full evaluation.
// ---------------------------------------------------------------------------
struct EmArgs {
    const void *feat;     // [K][H][W] pairs at storage precision
    const float *rho;     // [K][H][W] static prior of each ray
    const float *omr;     // [K][H][W] dynamic prior 1 - rho
    const float *mu_T;    // [H][W]
    float *q;             // [K][H][W], read at entry, written at exit
    int32_t *d_idx;       // [H][W], read at entry when seed_from_d, written at exit
    float *lpix;          // [H][W], objective of the last iteration
    double *obj;          // [n_iters][n_blocks] block sums of the objective
    int H, W, D, n_iters, n_blocks, tile, mode, seed_from_d;
    int want_obj;         // objective of every iteration (else only of the last)
    int dmin_i, dstep_i;  // integer levels (integer-shift path)
    float d_min, d_step;
    float beta_p;         // beta / K
    float beta;           // beta (enumeration modes: weight of the coupled variance)
    float lambda, gamma;
    float c_exp2;         // log2(e) / (2 sigma^2)
    float c_exp;          // 1 / (2 sigma^2)
    float prior_T;        // |d - mu| beyond which gamma + g == gamma in FP32
    float prior_hi;       // upper bound of the log prior as evaluated: ln(1 + gamma) plus slack
    float margin_k;       // one-pass error bound, in units of beta' * S
    float margin_c;       // absolute slack of the bound
    float win_half;       // > 0: the M-step searches only |d - mu| <= win_half
    int dyn_only;         // 1: only pixels with rho_ref < tau are reconstructed
    const int4 *items;    // dynamic-only work list: (row, first column, pixels, 0), or null for row tiles
    const int *n_items;   // its length (device)
    int seg_w;            // dynamic-only: columns an item's pixels may spread over (a multiple of 64, <= 256)
    float d_absmax;       // max |d_j| over the levels
    float inv_step;       // 1 / d_step
    float c_t2;           // 2 sigma^2 ln 2
    float tau;            // first-iteration threshold (dynamic-only test)
    unsigned long long *sweep_count;  // diagnostic, or null: level steps the sweeps take, summed over waves
    int perm[kMaxViews];  // kernel view order -> array view index (perm[0] = reference)
    int bi[kMaxViews];    // integer baselines, kernel order (integer-shift path)
    float b[kMaxViews];   // baselines, kernel order
};

// LDS record: descriptor pair at storage precision plus |f|^2 in FP32.
// Record format 3 holds FP32 descriptors exactly in 8 bytes: every descriptor
// is an integer Sobel response (|G| <= 3060) times 2^-12, kept as int16 G.
template <int ST> struct Rec;
template <> struct Rec<0> { using T = float4; };  // (Gx, Gy, |f|^2, unused)
template <> struct Rec<1> { using T = float2; };  // (half2 bits, |f|^2)
template <> struct Rec<2> { using T = float2; };  // (2 x bf16 bits, |f|^2)
template <> struct Rec<3> { using T = float2; };  // (2 x int16 G bits, |f|^2), f = G * 2^-12

template <int ST>
__device__ __forceinline__ typename Rec<ST>::T make_rec(typename Pair<ST>::T v) {
    const float2 f = widen(v);
    const float n = fmaf(f.x, f.x, f.y * f.y);
    if constexpr (ST == 0) return make_float4(f.x, f.y, n, 0.0f);
    else if constexpr (ST == 1) return make_float2(__uint_as_float(*reinterpret_cast<const uint32_t *>(&v)), n);
    else return make_float2(__uint_as_float(v), n);
}

template <int ST>
__device__ __forceinline__ float2 rec_f(const typename Rec<ST>::T &r) {
    if constexpr (ST == 0) return make_float2(r.x, r.y);
    else if constexpr (ST == 3) {
        // G * 2^-12 by an exponent shift, not a product: the compiler fuses
        // products with neighbouring additions, and the arithmetic after the
        // fetch must have the same shape (and bits) as with the other formats
        const uint32_t u = __float_as_uint(r.x);
        return make_float2(__builtin_amdgcn_ldexpf((float)(int16_t)(u & 0xffffu), -12),
                           __builtin_amdgcn_ldexpf((float)(int16_t)(u >> 16), -12));
    } else {
        const uint32_t u = __float_as_uint(r.x);
        if constexpr (ST == 1) return widen(*reinterpret_cast<const __half2 *>(&u));
        else return widen(u);
    }
}

template <int ST>
__device__ __forceinline__ float rec_n(const typename Rec<ST>::T &r) {
    if constexpr (ST == 0) return r.z;
    else return r.y;
}

// LDS window of one view for one row tile: positions umin .. umin+len-1 of
// the view's row (replicated border), one record each, consecutive.
struct Window {
    int umin, off, len;  // first staged position, offset in LDS (records), staged positions
};

template <int K, bool FRAC>
__device__ __forceinline__ void view_windows(const EmArgs &a, int x0, int tw, Window (&w)[K], int &total) {
    int off = 0;
    const float d_max = a.d_min + (float)(a.D - 1) * a.d_step;
    const int dmax_i = a.dmin_i + (a.D - 1) * a.dstep_i;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int umin, umax;
        if (FRAC) {
            const float s0 = a.b[k] * a.d_min, s1 = a.b[k] * d_max;
            umin = (int)floorf((float)x0 - fmaxf(s0, s1)) - 2;
            umax = (int)floorf((float)(x0 + tw - 1) - fminf(s0, s1)) + 3;
        } else {
            const int s0 = a.bi[k] * a.dmin_i, s1 = a.bi[k] * dmax_i;
            umin = x0 - max(s0, s1);
            umax = x0 + tw - 1 - min(s0, s1);
        }
        w[k].umin = umin;
        w[k].off = off;
        w[k].len = umax - umin + 1;
        off += w[k].len;
    }
    total = off;
}

// LDS record index of staged position p (0 <= p < len) of a window.
__device__ __forceinline__ int win_index(const Window &w, int p) { return w.off + p; }

// Record index of a lane's footprint at level 0 (integer shifts); level j is
// at that index - b_k * d_step * j.
__device__ __forceinline__ int lane_index0(const Window &w, int bi, int dmin_i, int x) {
    return win_index(w, x - bi * dmin_i - w.umin);
}

// Unit-spaced symmetric arrays (b_k = k - ref, ref = (K-1)/2, d_step = 1):
// the baseline of kernel view kk (kernel view 0 is the reference, the others
// follow in array order) is a compile-time constant.
template <int K>
__host__ __device__ constexpr int sym_baseline(int kk) {
    return kk == 0 ? 0 : ((kk - 1 < (K - 1) / 2 ? kk - 1 : kk) - (K - 1) / 2);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Descriptor (and |f|^2) of kernel view k at level j for pixel x; idx0 is
// the lane's level-0 record index of the view (integer shifts).
template <int K, int ST, bool FRAC>
__device__ __forceinline__ void fetch(const typename Rec<ST>::T *win, const Window &w, const EmArgs &a, int k,
                                      int x, int j, int idx0, float2 &f, float &n) {
    if (FRAC) {
        const float d = fmaf((float)j, a.d_step, a.d_min);
        int i0;
        float t;
        footprint(x, a.b[k], d, i0, t);
        // the window margins cover float rounding of the footprint; the
        // clamp keeps every read inside this view's window regardless
        const int p = clampi(w.off + i0 - w.umin, w.off, w.off + w.len - 2);
        const float2 v0 = rec_f<ST>(win[p]), v1 = rec_f<ST>(win[p + 1]);
        f = make_float2(lerp(v0.x, v1.x, t), lerp(v0.y, v1.y, t));
        n = fmaf(f.x, f.x, f.y * f.y);
    } else {
        const typename Rec<ST>::T r = win[idx0 - a.bi[k] * a.dstep_i * j];
        f = rec_f<ST>(r);
        n = rec_n<ST>(r);
    }
}

// Exact energy at one level, E = cw * C - logP: two-pass weighted mean and
// spread with the M-step weights wt, summed in kernel view order; shared by
// the exact re-evaluation and the exhaustive sweep so both give the same bits.
// With wt >= 0 and cw >= 0 the result is never below -P: C is a sum of
// non-negative terms and the fma rounds monotonically.
template <int K>
__device__ __forceinline__ float exact_energy(const float2 (&f)[K], const float (&wt)[K], float invW, float cw,
                                              float P, float &mx, float &my) {
    float ax = 0.0f, ay = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ax = fmaf(wt[k], f[k].x, ax);
        ay = fmaf(wt[k], f[k].y, ay);
    }
    mx = ax * invW;
    my = ay * invW;
    float C = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float dx = f[k].x - mx, dy = f[k].y - my;
        C = fmaf(wt[k], fmaf(dx, dx, dy * dy), C);
    }
    return fmaf(cw, C, -P);
}

// ln(gamma + exp(-(d_j - mu)^2 / (2 sigma^2))), the log disparity prior up to
// a constant, through the hardware base-2 exponential and logarithm.
__device__ __forceinline__ float log_prior(const EmArgs &a, int j, float mu) {
    const float t = fmaf((float)j, a.d_step, a.d_min) - mu;
    const float g = __builtin_amdgcn_exp2f(-(t * t) * a.c_exp2);
    return kLn2 * __builtin_amdgcn_logf(a.gamma + g);
}

// Log prior as the M-step sweep scores it: with a search window (masked),
// levels farther than win_half from mu are excluded (-inf).
__device__ __forceinline__ float sweep_log_prior(const EmArgs &a, int j, float mu, bool masked) {
    if (masked && fabsf(fmaf((float)j, a.d_step, a.d_min) - mu) > a.win_half) return -INFINITY;
    return log_prior(a, j, mu);
}

// Per-lane state of one pixel across EM iterations.
template <int K>
struct Lane {
    float q[K];    // weights (kernel view order)
    float la[K];   // ln rho_k + lambda
    float lb[K];   // ln(1 - rho_k)
    float2 f0;     // reference-view descriptor (constant over levels)
    float n0;      // its squared norm
    float mu;      // prior disparity
    float L;       // objective after the last E-step
    int best_j;    // level of the last M-step (seed of the next sweep)
    int c;         // level nearest mu (constant over the iterations)
    int idx0[K];   // level-0 LDS record index of each view (integer shifts)
};

// Levels swept per unrolled group: the group's records stay in registers.
template <int K>
constexpr int sweep_group() { return K - 1 <= 4 ? 4 : (K - 1 <= 8 ? 2 : 1); }

// Wave-uniform window [jlo, jhi] of levels where the log prior differs from
// the constant ln(gamma); outside it gamma + g rounds to gamma in FP32.
__device__ __forceinline__ void prior_window(const EmArgs &a, bool active, float mu, int &jlo, int &jhi) {
    jlo = a.D;
    jhi = -1;
    if (active) {
        // clamped in float before the conversion: mu far outside the level
        // range (or not finite, with the deferred input check) stays defined
        jlo = (int)fminf(fmaxf(ceilf((mu - a.prior_T - a.d_min) / a.d_step), 0.0f), (float)a.D);
        jhi = (int)fmaxf(fminf(floorf((mu + a.prior_T - a.d_min) / a.d_step), (float)(a.D - 1)), -1.0f);
    }
    // uniform across the wave: keep them in scalar registers
    jlo = __builtin_amdgcn_readfirstlane(wave_min(jlo));
    jhi = __builtin_amdgcn_readfirstlane(wave_max(jhi));
}

// The level nearest the prior disparity, clamped to the level range; a mu
// exactly half-way between two levels takes the lower one (the arg min's tie
// rule).  The quotient is formed in double from the single-precision mu,
// d_min and d_step, so a half-way point is seen exactly.  It decides the
// level of pixels that are not swept (dynamic-only, an empty search window)
// and seeds the first sweep.
__device__ __forceinline__ int nearest_level(const EmArgs &a, float mu) {
    const double t = ((double)mu - (double)a.d_min) / (double)a.d_step;
    return (int)fmin(fmax(ceil(t - 0.5), 0.0), (double)(a.D - 1));
}

constexpr float kLog2e = 1.44269504088896341f;

// E-step by enumeration of all 2^K labelings S of the pixel's rays (the
// enumeration modes, Sec. III-C last sentence and Sec. III-D): the log weight
// of S is sum_k ln P(S_k | rho_k) - beta Var_S, with Var_S the variance of
// the static descriptors normalised by their number (0 for fewer than two).
// f are the descriptors at the chosen level (kernel view order), (mx, my) the
// M-step mean: the descriptors enter centred on it (the variance does not
// change) so that the one-pass variance keeps its accuracy.  ENUM_SOFT sets
// q to the marginals P(S_k = 1), accumulated with weights scaled by the
// largest log weight so far; ENUM_HARD sets q to the labeling of largest
// weight, ties to the largest mask in array view order.  Returns the log of
// the summed weights (soft) or of the largest weight (hard).
template <int K>
__device__ __forceinline__ float enum_estep(const float2 (&f)[K], float mx, float my, const EmArgs &a, Lane<K> &s) {
    float gx[K], gy[K], gn[K], l1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        gx[k] = f[k].x - mx;
        gy[k] = f[k].y - my;
        gn[k] = fmaf(gx[k], gx[k], gy[k] * gy[k]);
        l1[k] = s.la[k] - a.lambda;   // ln rho_k
    }
    const bool hard = a.mode == 3;
    float top = -INFINITY, Z = 0.0f, acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0f;
    int best_amask = 0, best_mask = 0;
    for (int mask = 0; mask < (1 << K); ++mask) {
        float ax = 0.0f, ay = 0.0f, s2 = 0.0f, lw = 0.0f;
        int n = 0, amask = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool on = (mask >> k) & 1;
            ax += on ? gx[k] : 0.0f;
            ay += on ? gy[k] : 0.0f;
            s2 += on ? gn[k] : 0.0f;
            lw += on ? l1[k] : s.lb[k];
            n += on ? 1 : 0;
            amask |= on ? (1 << a.perm[k]) : 0;
        }
        if (n >= 2) {
            const float inv = 1.0f / (float)n;
            const float var = fmaxf(fmaf(-(ax * ax + ay * ay), inv, s2) * inv, 0.0f);
            lw = fmaf(-a.beta, var, lw);
        }
        if (hard) {
            if (lw > top || (lw == top && amask > best_amask)) {
                top = lw;
                best_amask = amask;
                best_mask = mask;
            }
        } else {
            const float mn = fmaxf(top, lw);
            if (mn > -INFINITY) {
                const float r = __builtin_amdgcn_exp2f((top - mn) * kLog2e);
                const float w = __builtin_amdgcn_exp2f((lw - mn) * kLog2e);
                Z = fmaf(Z, r, w);
#pragma unroll
                for (int k = 0; k < K; ++k) acc[k] = fmaf(acc[k], r, ((mask >> k) & 1) ? w : 0.0f);
                top = mn;
            }
        }
    }
    if (hard) {
#pragma unroll
        for (int k = 0; k < K; ++k) s.q[k] = ((best_mask >> k) & 1) ? 1.0f : 0.0f;
        return top;
    }
    // a true division: a view static in every weighted labeling gets exactly 1
#pragma unroll
    for (int k = 0; k < K; ++k) s.q[k] = acc[k] / Z;
    return top + kLn2 * __builtin_amdgcn_logf(Z);
}

// Levels a lane's M-step searches: all of them, or those within win_half of
// the prior disparity (the level nearest it when none is).
__device__ __forceinline__ void search_window(const EmArgs &a, float mu, int &wlo, int &whi) {
    wlo = 0;
    whi = a.D - 1;
    if (a.win_half > 0.0f) {
        const float lo = ceilf((mu - a.win_half - a.d_min) / a.d_step);
        const float hi = floorf((mu + a.win_half - a.d_min) / a.d_step);
        wlo = (int)fminf(fmaxf(lo, 0.0f), (float)(a.D - 1));
        whi = (int)fmaxf(fminf(hi, (float)(a.D - 1)), 0.0f);
        if (!(lo <= (float)(a.D - 1)) || !(hi >= 0.0f) || lo > hi) wlo = whi = nearest_level(a, mu);
    }
}

// Union [slo, shi] of the search windows of the wave's working lanes
// (uniform).  Within it the sweep excludes a lane's other levels through its
// prior (sweep_log_prior).
__device__ __forceinline__ void search_range(const EmArgs &a, bool work, float mu, int &slo, int &shi) {
    int wlo, whi;
    search_window(a, mu, wlo, whi);
    slo = __builtin_amdgcn_readfirstlane(wave_min(work ? wlo : a.D));
    shi = __builtin_amdgcn_readfirstlane(wave_max(work ? whi : -1));
}

// M-step weights of one pixel (Eq. 6): the posteriors q_k, or all 1 when none
// is positive (then the spread term is dropped, cw = 0); invW = 1 / sum wt.
template <int K>
__device__ __forceinline__ void mstep_weights(const EmArgs &a, const float (&q)[K], float (&wt)[K], float &invW,
                                              float &cw) {
    float Q = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) Q += q[k];
    const bool empty = !(Q > 0.0f);
#pragma unroll
    for (int k = 0; k < K; ++k) wt[k] = empty ? 1.0f : q[k];
    // hardware reciprocal (1 ulp): the exact energies of the fast and the
    // exhaustive sweep both use this value
    invW = __builtin_amdgcn_rcpf(empty ? (float)K : Q);
    cw = empty ? 0.0f : a.beta_p;
}

// Level-0 LDS record index of each of a pixel's footprints (integer shifts).
template <int K, bool FRAC>
__device__ __forceinline__ void level0_index(const Window (&w)[K], const EmArgs &a, int x, int (&idx0)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) idx0[k] = FRAC ? 0 : lane_index0(w[k], a.bi[k], a.dmin_i, x);
}

// Exact M-step energy of one pixel at level j.
template <int K, int ST, bool FRAC>
__device__ __forceinline__ float level_energy(const typename Rec<ST>::T *win, const Window (&w)[K], const EmArgs &a,
                                              int x, const int (&idx0)[K], float2 f0, int j, const float (&wt)[K],
                                              float invW, float cw, float mu, bool masked) {
    float2 f[K];
    float nn, mx, my;
    f[0] = f0;
#pragma unroll
    for (int k = 1; k < K; ++k) fetch<K, ST, FRAC>(win, w[k], a, k, x, j, idx0[k], f[k], nn);
    return exact_energy<K>(f, wt, invW, cw, sweep_log_prior(a, j, mu, masked), mx, my);
}

// Fast M-step sweep of one pixel over levels jbase + [lo, hi): those in
// jbase + [j1, j2) with the prior evaluated lazily, the others with the
// constant ln gamma (levels outside the prior window).  ib[k] is the LDS
// record index of view k at level jbase (integer shifts).  best_E and best_j
// enter as the seed level and its exact energy and leave as the minimum,
// ties to the lowest level.
template <int K, int ST, bool FRAC, bool SYM>
__device__ __forceinline__ void fast_sweep(const typename Rec<ST>::T *win, const Window (&w)[K], const EmArgs &a,
                                           int x, const int (&ib)[K], int jbase, int lo, int j1, int j2, int hi,
                                           float Pc, float phi, const float (&wt)[K], float invW, float cw, float2 f0,
                                           float n0, float mu, bool masked, float &best_E, int &best_j) {
    using R = typename Rec<ST>::T;
    // candidate test  E^ - M <= E_best  with the margin folded in:
    //   cw (1 - margin_k) S - (cw / W) |A|^2  <=  E_best + margin_c + P_j,
    // evaluated with the weights pre-scaled by sg = sqrt(cw / W), so that
    // |A'|^2 = (cw / W) |A|^2 and S' = sg S, as c3 S' - |A'|^2 with
    // c3 = cw (1 - margin_k) / sg (the extra roundings stay well inside
    // margin_k's slack)
    // hardware square root and reciprocal: c3 * sg is cw (1 - margin_k)
    // to a few ulps, far inside margin_k's slack
    const float sg = __builtin_amdgcn_sqrtf(cw * invW);
    const float c3 = sg > 0.0f ? cw * (1.0f - a.margin_k) * __builtin_amdgcn_rcpf(sg) : 0.0f;
    float ws[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ws[k] = sg * wt[k];
    const float A0x = ws[0] * f0.x, A0y = ws[0] * f0.y, S0 = ws[0] * n0;
    float bound = best_E + a.margin_c;
    float bound_c = bound + Pc;            // threshold where the prior is the constant ln gamma
    float bound_hi = bound + phi;          // threshold with the prior's upper bound over the levels
    // Scores G consecutive levels from jbase + j0, then re-evaluates the
    // candidates among them exactly, in increasing level order.
    auto group = [&](auto Gc, int j0, bool inwin) {
        constexpr int G = decltype(Gc)::value;
        float2 f[G][K];
        float lhs[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            f[i][0] = f0;
            float ax = A0x, ay = A0y, S = S0;
#pragma unroll
            for (int k = 1; k < K; ++k) {
                float n;
                if constexpr (FRAC) {
                    fetch<K, ST, FRAC>(win, w[k], a, k, x, jbase + j0 + i, 0, f[i][k], n);
                } else if constexpr (SYM) {
                    // compile-time step per level: immediate LDS offsets
                    const int b = sym_baseline<K>(k);   // folds once k is unrolled
                    const R *base = win + ib[k] - b * (b > 0 ? j0 + G - 1 : j0);
                    const R r = base[b > 0 ? b * (G - 1 - i) : -b * i];
                    f[i][k] = rec_f<ST>(r);
                    n = rec_n<ST>(r);
                } else {
                    const R r = win[ib[k] - a.bi[k] * a.dstep_i * (j0 + i)];
                    f[i][k] = rec_f<ST>(r);
                    n = rec_n<ST>(r);
                }
                ax = fmaf(ws[k], f[i][k].x, ax);
                ay = fmaf(ws[k], f[i][k].y, ay);
                S = fmaf(ws[k], n, S);
            }
            lhs[i] = fmaf(c3, S, -fmaf(ax, ax, ay * ay));
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int j = jbase + j0 + i;
            // Inside the prior window the prior is evaluated only for
            // levels that pass the test with its upper bound P_hi (few:
            // the seed is close to the optimum); the current best level
            // is already exact and is skipped.
            float Pj = Pc;
            bool cand;
            if (inwin) {
                cand = false;
                if (lhs[i] <= bound_hi) {
                    Pj = sweep_log_prior(a, j, mu, masked);
                    cand = lhs[i] <= bound + Pj;
                }
            } else {
                cand = lhs[i] <= bound_c;
            }
            if (cand && j != best_j) {
                float mx, my;
                const float E = exact_energy<K>(f[i], wt, invW, cw, Pj, mx, my);
                if (E < best_E || (E == best_E && j < best_j)) {
                    best_E = E;
                    best_j = j;
                    bound = best_E + a.margin_c;
                    bound_c = bound + Pc;
                    bound_hi = bound + phi;
                }
            }
        }
    };
    constexpr int G = sweep_group<K>();
    auto sweep = [&](int jb, int je, bool inwin) {
        int j = jb;
        for (; j + G <= je; j += G) group(std::integral_constant<int, G>{}, j, inwin);
        for (; j < je; ++j) group(std::integral_constant<int, 1>{}, j, inwin);
    };
    sweep(lo, j1, false);
    sweep(j1, j2, true);
    sweep(j2, hi, false);
}

// E-step (Eq. 7) of one pixel at level j with the M-step weights wt: the
// static posterior of each ray (or the enumeration E-step) and, with_obj,
// the pixel's objective.
template <int K, int ST, bool FRAC>
__device__ __forceinline__ void estep(const typename Rec<ST>::T *win, const Window (&w)[K], const EmArgs &a, int x,
                                      const int (&idx0)[K], float2 f0, int j, const float (&wt)[K], float invW,
                                      float cw, Lane<K> &s, bool with_obj) {
    float2 f[K];
    float nn, mx, my;
    f[0] = f0;
#pragma unroll
    for (int k = 1; k < K; ++k) fetch<K, ST, FRAC>(win, w[k], a, k, x, j, idx0[k], f[k], nn);
    (void)exact_energy<K>(f, wt, invW, cw, 0.0f, mx, my);
    float L = 0.0f;
    if (with_obj) L = log_prior(a, j, s.mu);
    if (a.mode >= 2) {
        s.L = L + enum_estep<K>(f, mx, my, a, s);
        return;
    }
    // posterior in the logit domain with the hardware base-2 exponential and
    // reciprocal (about 1e-7 absolute error; q = 0 or 1 exactly at +-inf)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float dx = f[k].x - mx, dy = f[k].y - my;
        const float e = fmaf(dx, dx, dy * dy);
        const float a1 = s.la[k] - a.beta_p * e;
        const float a0 = s.lb[k];
        if (a.mode == 1) {
            s.q[k] = (a1 >= a0) ? 1.0f : 0.0f;
            if (with_obj) L += fmaxf(a1, a0);
        } else {
            s.q[k] = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f((a0 - a1) * kLog2e));
            if (with_obj) {
                // logaddexp(a1, a0) = max + ln(1 + exp(-|a1 - a0|))
                const float r = __builtin_amdgcn_exp2f(-fabsf(a1 - a0) * kLog2e);
                L += fmaxf(a1, a0) + kLn2 * __builtin_amdgcn_logf(1.0f + r);
            }
        }
    }
    s.L = L;
}

// Sweep range of the levels the prior window splits [slo, shi] into: below,
// inside [j1, j2) and above it (a lane's search window lies inside its prior
// window).
__device__ __forceinline__ void window_split(int jlo, int jhi, int slo, int shi, int &lo, int &j1, int &j2, int &hi) {
    lo = slo;
    hi = shi + 1;
    j1 = min(max(jlo, lo), hi);
    j2 = min(max(jhi + 1, j1), hi);
}

// One EM iteration of one active lane: M-step sweep over all levels with the
// current weights, then the E-step and the objective at the chosen level.
// [jlo, jhi] is the wave's prior window and [slo, shi] the union of its
// lanes' search windows.
template <int K, int ST, bool FRAC, bool EXH, bool SYM>
__device__ __forceinline__ void em_iteration(const typename Rec<ST>::T *win, const Window (&w)[K], const EmArgs &a,
                                             int x, int jlo, int jhi, int slo, int shi, float Pc, Lane<K> &s,
                                             bool with_obj) {
    float wt[K], invW, cw;
    mstep_weights<K>(a, s.q, wt, invW, cw);
    const float mu = s.mu;
    int best_j = s.best_j;
    const bool masked = a.win_half > 0.0f;   // uniform: search window set
    if (EXH) {
        // keeps the seed only when no level of the lane's window has a finite
        // energy, i.e. when the window is empty and the seed is its fallback
        float best_E = INFINITY;
        for (int j = slo; j <= shi; ++j) {
            const float E = level_energy<K, ST, FRAC>(win, w, a, x, s.idx0, s.f0, j, wt, invW, cw, mu, masked);
            if (E < best_E) {
                best_E = E;
                best_j = j;
            }
        }
    } else {
        // seed: exact energy at the previous level
        float best_E = level_energy<K, ST, FRAC>(win, w, a, x, s.idx0, s.f0, best_j, wt, invW, cw, mu, masked);
        int lo, j1, j2, hi;
        window_split(jlo, jhi, slo, shi, lo, j1, j2, hi);
        fast_sweep<K, ST, FRAC, SYM>(win, w, a, x, s.idx0, 0, lo, j1, j2, hi, Pc, a.prior_hi, wt, invW, cw, s.f0,
                                     s.n0, mu, masked, best_E, best_j);
    }
    s.best_j = best_j;
    estep<K, ST, FRAC>(win, w, a, x, s.idx0, s.f0, best_j, wt, invW, cw, s, with_obj);
}

// Levels that can still win under the prior bound of the M-step (Eq. 6):
// the energy E_j = cw C_j - P_j of a level is never below -P_j (C_j >= 0,
// see exact_energy), so a level whose log prior P_j, as the kernel
// evaluates it, is below -E_best can neither beat nor tie the best energy
// found so far.  P_j falls off with |d_j - mu|, so the levels that remain
// form an interval [jl, jh] around mu; returns false when the bound excludes
// nothing (E_best not below -ln gamma, or not finite).  The slacks cover
// the error of the evaluated prior (hardware exp2 and log2 and the rounding
// of (d_j - mu)^2 c: under 2e-5 relative on the exponential, 1e-5 (1 + |P|)
// on P), of this function's own hardware exp2, log2 and square root, and
// the rounding of d_j - mu and of the level position of mu.
__device__ __forceinline__ bool prior_interval(const EmArgs &a, float best_E, float mu, int &jl, int &jh) {
    const float tgt = -best_E - 1e-5f * (1.0f + fabsf(best_E));
    // lower bound of exp(tgt) - gamma (the subtraction is exact while
    // exp(tgt) <= 2 gamma)
    const float G = __builtin_amdgcn_exp2f(tgt * kLog2e) * (1.0f - 0x1p-16f) - a.gamma;
    if (!(G > 0.0f)) return false;
    // exp(-t^2 / (2 sigma^2)) < G (1 - 1e-4) for |t| > tmax, where
    // tmax^2 = -ln(G (1 - 1e-4)) 2 sigma^2 = -log2(G (1 - 1e-4)) 2 sigma^2 ln 2
    const float l2 = __builtin_amdgcn_logf(fminf(G * (1.0f - 1e-4f), 1.0f));
    const float tmax = __builtin_amdgcn_sqrtf(fmaxf(-l2, 0.0f) * a.c_t2) * (1.0f + 1e-4f) +
                       0x1p-20f * (a.d_absmax + fabsf(mu));
    const float m = (mu - a.d_min) * a.inv_step, r = tmax * a.inv_step;
    // clamped to [0, D] and [-1, D - 1] before the conversion, so that a
    // position far outside the level range converts exactly
    jl = (int)fminf(fmaxf(ceilf(m - r - 0.01f), 0.0f), (float)a.D);
    jh = (int)fmaxf(fminf(floorf(m + r + 0.01f), (float)(a.D - 1)), -1.0f);
    return true;
}

// (E, j) <- the smaller of (E, j) and (E2, j2) in the sweep's order: lower
// energy, then lower level.
__device__ __forceinline__ void lex_min(float &E, int &j, float E2, int j2) {
    if (E2 < E || (E2 == E && j2 < j)) {
        E = E2;
        j = j2;
    }
}

// Position of the u-th set bit (u counted from 0) of a 64-bit mask with more
// than u set bits.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int u) {
    int pos = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int p = pos + step;
        if (__popcll(m & ((1ull << p) - 1ull)) <= u) pos = p;
    }
    return pos;
}

// Sweep overhead of handing a pixel's levels to other lanes, in levels.
constexpr int kShareCost = 6;

// M-step sweep of a kernel instance: the fast sweep with the prior bound and
// the wave's lanes sharing levels (integer shifts), the exhaustive sweep, or
// the fast sweep of each lane on its own (fractional shifts, and search
// windows: their short ranges gain too little to pay for the bound).
constexpr int kSweepShared = 0, kSweepExhaustive = 1, kSweepLane = 2;

// One EM iteration of one wave with the M-step work rebalanced inside the
// wave (integer shifts, fast sweep, no search window: the levels excluded by
// a window would be swept, to no effect).  Each pixel's seed energy bounds the
// levels that can still win (prior_interval).  A wave sweeps until its
// slowest lane is done, so instead of every lane sweeping its own levels:
//   * pixels with a bounded interval sweep a window of the wave's widest
//     interval, placed over their own;
//   * the levels of the pixels the bound leaves unbounded are cut into cp
//     chunks each (cp a power of two, cp * n_unbounded <= 64), one chunk per
//     lane: the pixel's M-step inputs come over by lane shuffles, each chunk
//     is swept from the pixel's seed, and the chunk results are reduced
//     back with the sweep's order (lower energy, then lower level).
// The wave does this when it takes fewer levels than one full sweep, else
// every lane sweeps its whole range.  The levels excluded cannot be the
// minimum and the reduction keeps the tie rule, so the result is the full
// sweep's, bit for bit.
// x_idle is a column inside every view's window (the tile's first), read by
// lanes without a pixel.  Returns the number of level steps the wave's sweep
// takes (uniform; diagnostics).
template <int K, int ST, bool SYM>
__device__ __forceinline__ int shared_iteration(const typename Rec<ST>::T *win, const Window (&w)[K],
                                                 const EmArgs &a, int x, int x_idle, bool work, int jlo, int jhi,
                                                 int slo, int shi, float Pc, Lane<K> &s, bool with_obj) {
    using R = typename Rec<ST>::T;
    const int lane = threadIdx.x & 63;
    const bool masked = a.win_half > 0.0f;

    float wt[K], invW = 0.0f, cw = 0.0f, best_E = INFINITY;
    int best_j = s.best_j;
    int idx0[K];
    level0_index<K, false>(w, a, work ? x : x_idle, idx0);
    const R r0 = win[idx0[0]];
    const float2 f0 = rec_f<ST>(r0);
    const float n0 = rec_n<ST>(r0);
    int jl = 0, jh = -1;
    bool bnd = false;
    if (work) {
        mstep_weights<K>(a, s.q, wt, invW, cw);
        best_E = level_energy<K, ST, false>(win, w, a, x, idx0, f0, best_j, wt, invW, cw, s.mu, masked);
        bnd = prior_interval(a, best_E, s.mu, jl, jh);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) wt[k] = 0.0f;
    }
    const bool unb = work && !bnd;
    const uint64_t um = __ballot(unb);
    const int nu = __popcll(um);
    const bool anyb = __ballot(bnd) != 0;
    // no search window here: every lane searches all D levels
    const int nlev = a.D;
    // bounded windows: the wave's widest extents below and above each lane's
    // nearest level c to mu, so that neighbouring lanes (whose c mostly
    // agree) read neighbouring LDS records
    const int c = s.c;
    const int el = __builtin_amdgcn_readfirstlane(wave_max(bnd ? max(c - jl, 0) : 0));
    const int er = __builtin_amdgcn_readfirstlane(wave_max(bnd ? max(jh - c, 0) : 0));
    const int wl = el + er + 1;
    int cp = 1;
    while (nu > 0 && cp * 2 * nu <= 64) cp *= 2;
    // odd chunk lengths: the cp chunks of a pixel then start on different
    // LDS banks
    const int chunk = min(((nlev + cp - 1) / cp) | 1, nlev);
    const int cost = (anyb ? wl : 0) + (nu > 0 ? chunk + kShareCost : 0);
    const int steps = cost >= nlev ? max(shi - slo + 1, 0) : (anyb ? wl : 0) + (nu > 0 ? chunk : 0);

    if (cost >= nlev) {
        // every lane sweeps its whole range
        if (work) {
            int lo, j1, j2, hi;
            window_split(jlo, jhi, slo, shi, lo, j1, j2, hi);
            fast_sweep<K, ST, false, SYM>(win, w, a, x, idx0, 0, lo, j1, j2, hi, Pc, a.prior_hi, wt, invW, cw, f0,
                                          n0, s.mu, masked, best_E, best_j);
        }
    } else {
        // bounded pixels: wl levels from js, covering [jl, jh], inside the range
        if (anyb) {
            const int js = min(max(c - el, 0), a.D - wl);
            int ib[K];
#pragma unroll
            for (int k = 0; k < K; ++k) ib[k] = idx0[k] - a.bi[k] * a.dstep_i * js;
            if (bnd)
                fast_sweep<K, ST, false, SYM>(win, w, a, x, ib, js, 0, 0, wl, wl, Pc, a.prior_hi, wt, invW, cw, f0, n0,
                                              s.mu, masked, best_E, best_j);
        }
        // unbounded pixels: with U = 64 / cp, lane h sweeps chunk h / U of
        // the (h % U)-th one, so that the lanes sweeping the same chunk of
        // neighbouring pixels read neighbouring LDS records
        if (nu > 0) {
            const int U = 64 / cp;
            const int u = lane & (U - 1);
            const bool helper = u < nu;
            const int src = nth_set_bit(um, helper ? u : 0);
            float hwt[K];
#pragma unroll
            for (int k = 0; k < K; ++k) hwt[k] = __shfl(wt[k], src, 64);
            const float hinvW = __shfl(invW, src, 64), hcw = __shfl(cw, src, 64), hmu = __shfl(s.mu, src, 64);
            const int hc = __shfl(s.c, src, 64);
            float hE = __shfl(best_E, src, 64);
            int hj = __shfl(best_j, src, 64);
            // every shuffle runs on the whole wave: a lane shuffle reads
            // nothing from lanes switched off by a branch
            const int xs = __shfl(x, src, 64);
            const int hx = helper ? xs : x_idle;
            int hidx0[K];
            level0_index<K, false>(w, a, hx, hidx0);
            const R hr0 = win[hidx0[0]];
            const int jb = min((lane / U) * chunk, a.D - chunk);
            // upper bound of the prior over the chunk: its value at the
            // chunk's level nearest mu, plus the evaluation's error
            const int jn = min(max(hc, jb), jb + chunk - 1);
            const float pn = log_prior(a, jn, hmu);
            const float phi = pn + 1e-5f * (1.0f + fabsf(pn));
            int ib[K];
#pragma unroll
            for (int k = 0; k < K; ++k) ib[k] = hidx0[k] - a.bi[k] * a.dstep_i * jb;
            if (helper)
                fast_sweep<K, ST, false, SYM>(win, w, a, hx, ib, jb, 0, 0, chunk, chunk, Pc, phi, hwt, hinvW, hcw,
                                              rec_f<ST>(hr0), rec_n<ST>(hr0), hmu, masked, hE, hj);
            // reduce each pixel's cp chunks (lanes u, u + U, u + 2U, ...)
            for (int o = U; o < 64; o <<= 1) {
                const float E2 = __shfl_xor(hE, o, 64);
                const int j2 = __shfl_xor(hj, o, 64);
                lex_min(hE, hj, E2, j2);
            }
            const int rank = __popcll(um & ((1ull << lane) - 1ull));
            const int jr = __shfl(hj, unb ? rank : 0, 64);
            if (unb) best_j = jr;
        }
    }
    s.best_j = best_j;
    if (work) {
        // the E-step's inputs again (the same bits): cheaper than keeping
        // them live through the sweeps
        float wt2[K], invW2, cw2;
        mstep_weights<K>(a, s.q, wt2, invW2, cw2);
        int idx2[K];
        level0_index<K, false>(w, a, x, idx2);
        estep<K, ST, false>(win, w, a, x, idx2, rec_f<ST>(win[idx2[0]]), best_j, wt2, invW2, cw2, s, with_obj);
    }
    return steps;
}

// Descriptor pair of storage ST as a pair of record storage RS (RS == ST,
// or FP32 values already known to be exact in binary16).
template <int RS, int ST>
__device__ __forceinline__ typename Pair<RS>::T to_record_pair(typename Pair<ST>::T v) {
    if constexpr (RS == ST) return v;
    else {
        const float2 f = widen(v);
        return make_pair<RS>(f.x, f.y);
    }
}

__device__ __forceinline__ bool exact_in_half(float v) { return __half2float(__float2half_rn(v)) == v; }

// LDS record of a descriptor pair of storage ST in record format RS (RS ==
// ST; FP32 values exact in binary16 as RS = 1; any FP32 values as RS = 3).
template <int RS, int ST>
__device__ __forceinline__ typename Rec<RS>::T stage_rec(typename Pair<ST>::T v) {
    if constexpr (RS == 3) {
        const float2 f = widen(v);
        const int gx = (int)(f.x * 4096.0f), gy = (int)(f.y * 4096.0f);   // exact: |G| <= 3060
        const uint32_t bits = ((uint32_t)gx & 0xffffu) | ((uint32_t)gy << 16);
        return make_float2(__uint_as_float(bits), fmaf(f.x, f.x, f.y * f.y));
    } else {
        return make_rec<RS>(to_record_pair<RS, ST>(v));
    }
}

// The kernel body: descriptors of storage ST staged as records of storage RS.
// STAGED: the caller has staged the windows already (and synchronised).
template <int K, int ST, int RS, bool FRAC, int SW, bool SYM, bool STAGED = false>
__device__ __forceinline__ void em_body(const EmArgs &a, unsigned char *lds_raw, double *red, int y, int x0, int tw,
                                        int xc, int block_id) {
    using R = typename Rec<RS>::T;
    using P = typename Pair<ST>::T;
    R *win = reinterpret_cast<R *>(lds_raw);

    const int tid = threadIdx.x;
    const size_t HW = (size_t)a.H * a.W;

    Window w[K];
    int total;
    view_windows<K, FRAC>(a, x0, tw, w, total);

    // Stage the windows (replicated border outside the image) with |f|^2.
    if constexpr (!STAGED) {
        const P *feat = reinterpret_cast<const P *>(a.feat);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const P *row = feat + ((size_t)a.perm[k] * a.H + y) * a.W;
#pragma unroll 4
            for (int p = tid; p < w[k].len; p += blockDim.x)
                win[win_index(w[k], p)] = stage_rec<RS, ST>(row[clampi(w[k].umin + p, 0, a.W - 1)]);
        }
        __syncthreads();
    }
    // the lane's pixel x0 + xc (xc < 0: none); with dynamic-only every
    // pixel of the work list is reconstructed
    const int x = x0 + xc;
    const bool active = xc >= 0 && x < a.W;
    const size_t pix = (size_t)y * a.W + (active ? x : 0);

    Lane<K> s;
    s.mu = 0.0f;
    s.L = 0.0f;
    s.best_j = 0;
    s.c = 0;
    s.f0 = make_float2(0.0f, 0.0f);
    s.n0 = 0.0f;
    bool work = active;   // pixel reconstructed (all of them unless dynamic-only)
    if (active) {
        s.mu = a.mu_T[pix];
        s.c = nearest_level(a, s.mu);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t i = (size_t)a.perm[k] * HW + pix;
            const float r = a.rho[i], om = a.omr[i];
            s.q[k] = a.q[i];
            s.la[k] = (r > 0.0f ? logf(r) : -INFINITY) + a.lambda;   // ln rho + lambda
            s.lb[k] = (om > 0.0f ? logf(om) : -INFINITY);            // ln(1 - rho)
        }
        s.best_j = (a.seed_from_d && work) ? a.d_idx[pix] : s.c;
#pragma unroll
        for (int k = 0; k < K; ++k) s.idx0[k] = FRAC ? 0 : lane_index0(w[k], a.bi[k], a.dmin_i, x);
        fetch<K, RS, FRAC>(win, w[0], a, 0, x, 0, s.idx0[0], s.f0, s.n0);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) s.q[k] = s.la[k] = s.lb[k] = 0.0f;
    }

    const float Pc = kLn2 * __builtin_amdgcn_logf(a.gamma);
    int jlo, jhi, slo, shi;
    prior_window(a, work, s.mu, jlo, jhi);
    search_range(a, work, s.mu, slo, shi);

    unsigned long long steps = 0;   // level steps of this wave's sweeps (diagnostics)
    const bool any_work = __ballot(work) != 0;
    for (int it = 0; it < a.n_iters; ++it) {
        const bool with_obj = a.want_obj || it == a.n_iters - 1;
        if constexpr (SW == kSweepShared && !FRAC) {
            steps += shared_iteration<K, RS, SYM>(win, w, a, x, x0, work, jlo, jhi, slo, shi, Pc, s, with_obj);
        } else {
            if (work)
                em_iteration<K, RS, FRAC, SW == kSweepExhaustive, SYM>(win, w, a, x, jlo, jhi, slo, shi, Pc, s,
                                                                        with_obj);
            steps += any_work ? max(shi - slo + 1, 0) : 0;
        }
        if (!with_obj) continue;
        // ---- FP64 block sum of the objective ----
        double sum = wave_sum(work ? (double)s.L : 0.0);
        const int lane = tid & 63, wv = tid >> 6;
        if (lane == 0) red[wv] = sum;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) tot += red[i];
            a.obj[(size_t)it * a.n_blocks + block_id] = tot;
        }
        __syncthreads();
    }
    if (a.sweep_count && (tid & 63) == 0) atomicAdd(a.sweep_count, steps);
    if (active && a.n_iters > 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) a.q[(size_t)a.perm[k] * HW + pix] = s.q[k];
        a.d_idx[pix] = s.best_j;
        a.lpix[pix] = s.L;
    }
}

// EM kernel.  FP32 descriptors whose staged windows are all exact in
// binary16 (|G| <= 2048 for the Sobel responses, the usual case) are staged
// as binary16 records, the others as int16 Sobel responses: the same values
// in 8 bytes per record either way, and the same FP32 arithmetic, so the
// results are the same bits.  The windows are staged as binary16 while their
// values are checked, and staged again as int16 only when one is not exact.
template <int K, int ST, bool FRAC, int SW, bool SYM>
__device__ __forceinline__ void em_entry(const EmArgs &a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double red[8];
    __shared__ int slots[64];
    int y, x0, tw, xc, block_id;
    if (a.items) {
        // dynamic-only work item (one wave): the item's first up to 64
        // dynamic reference pixels (rho_ref < tau) of a row from its first
        // column on, within seg_w columns of it, one per lane; the tile
        // spans the first to the last of them
        // Blocks go to the XCDs round robin (block b to XCD b % 8): the
        // list's items (in row order) are dealt so that consecutive ones,
        // which stage overlapping windows of a row, run on one XCD and share
        // its L2 (the grid is a multiple of 8 and at least the list's bound).
        const int lin = blockIdx.x, n_items = *a.n_items;
        if (lin >= n_items && lin < a.n_blocks && threadIdx.x == 0) {
            // the objective partials past the list are zero
            for (int it = 0; it < a.n_iters; ++it)
                if (a.want_obj || it == a.n_iters - 1) a.obj[(size_t)it * a.n_blocks + lin] = 0.0;
        }
        const int per = (n_items + 7) >> 3;
        block_id = (lin & 7) * per + (lin >> 3);
        if ((lin >> 3) >= per || block_id >= n_items) return;
        const int4 item = a.items[block_id];
        y = item.x;
        const int first = item.y, take = max(min(item.z, 64), 1), lane = threadIdx.x;
        const float *rho_ref = a.rho + (size_t)a.perm[0] * a.H * a.W + (size_t)y * a.W;
        int before = 0;
        for (int c = 0; c < a.seg_w; c += 64) {
            const int col = first + c + lane;
            const bool dyn = col < a.W && rho_ref[col] < a.tau;
            const uint64_t m = __ballot(dyn);
            const int rank = before + __popcll(m & ((1ull << lane) - 1ull));
            if (dyn && rank < take) slots[rank] = col;
            before += __popcll(m);
        }
        const int cnt = min(before, take);   // >= 1: the first column is dynamic
        __syncthreads();
        x0 = slots[0];
        tw = slots[cnt - 1] - x0 + 1;
        xc = lane < cnt ? slots[lane] - x0 : -1;
    } else {
        // row tile.  Blocks go to the 8 XCDs round robin (block lin to XCD
        // lin % 8), each with its own L2, and the tiles of a row stage
        // overlapping halo windows: so a row's tiles all go to one XCD (rows
        // y with the same y mod 8 share one), in row order, and a tile's
        // halo hits in the L2 its neighbours filled.  Rows past the last
        // whole group of 8 keep the grid order.
        const int gx = (int)gridDim.x, lin = (int)blockIdx.y * gx + (int)blockIdx.x;
        int t = lin;
        if (lin < ((int)gridDim.y / 8) * 8 * gx) {
            const int k = lin >> 3;
            t = ((lin & 7) + 8 * (k / gx)) * gx + k % gx;
        }
        y = t / gx;
        x0 = (t - y * gx) * a.tile;
        tw = a.tile;
        xc = threadIdx.x;
        block_id = t;
    }
    if constexpr (ST == 0) {
        Window w[K];
        int total;
        view_windows<K, FRAC>(a, x0, tw, w, total);
        const float2 *feat = reinterpret_cast<const float2 *>(a.feat);
        typename Rec<1>::T *win = reinterpret_cast<typename Rec<1>::T *>(lds_raw);
        bool exact = true;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float2 *row = feat + ((size_t)a.perm[k] * a.H + y) * a.W;
#pragma unroll 4
            for (int p = threadIdx.x; p < w[k].len; p += blockDim.x) {
                const float2 v = row[clampi(w[k].umin + p, 0, a.W - 1)];
                exact = exact && exact_in_half(v.x) && exact_in_half(v.y);
                win[win_index(w[k], p)] = stage_rec<1, 0>(v);
            }
        }
        // (each lane restages its own positions, so no barrier is needed
        // between the two stagings)
        if (__syncthreads_and(exact))
            em_body<K, 0, 1, FRAC, SW, SYM, true>(a, lds_raw, red, y, x0, tw, xc, block_id);
        else
            em_body<K, 0, 3, FRAC, SW, SYM>(a, lds_raw, red, y, x0, tw, xc, block_id);
    } else {
        em_body<K, ST, ST, FRAC, SW, SYM>(a, lds_raw, red, y, x0, tw, xc, block_id);
    }
}

template <int K, int ST, bool FRAC, int SW, bool SYM>
__global__ __launch_bounds__(256) void lf_em_kernel(EmArgs a) {
    em_entry<K, ST, FRAC, SW, SYM>(a);
}

// The same kernel held to 168 VGPRs, three waves per SIMD (views 7 to 9).
template <int K, int ST, bool FRAC, int SW, bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void lf_em_kernel_w3(EmArgs a) {
    em_entry<K, ST, FRAC, SW, SYM>(a);
}

// The same kernel held to 96 VGPRs, five waves per SIMD (up to 5 views).
template <int K, int ST, bool FRAC, int SW, bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void lf_em_kernel_w5(EmArgs a) {
    em_entry<K, ST, FRAC, SW, SYM>(a);
}

// The same kernel held to 128 VGPRs, four waves per SIMD: for small view
// counts this costs a few spills outside the sweep and gains a wave of
// latency hiding (the sweep alternates LDS reads and FMAs).
template <int K, int ST, bool FRAC, int SW, bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void lf_em_kernel_w4(EmArgs a) {
    em_entry<K, ST, FRAC, SW, SYM>(a);
}

}  // namespace lfem
