// Device code of the EM static-background reconstruction for gfx950.
//
// Each kernel is one step of the per-pixel method (Sec. III-F: every pixel is
// processed independently):
//   lf_descriptors_kernel  3x3 Sobel responses of R+G+B (Sec. III-C)
//   lf_ray_prior_kernel    S_P of each view at the ray footprint of mu_T and the
//                          thresholded first weights (Sec. III-B, III-F)
//   lf_em_kernel           n EM iterations: M-step sweep over all disparity
//                          levels (Eq. 6, E(d)), E-step posterior (Eq. 7),
//                          per-pixel objective and its FP64 block sums
//   lf_refocus_kernel      mean of the static rays (Eq. 2)
//   lf_median3_kernel      3x3 per-channel median of the refocused image (Sec. III-E)
//
// A rectified linear array shifts views along x only, so the EM kernel stages
// one row tile of every view plus its disparity halo in LDS once per launch
// and sweeps all levels and iterations from there; one lane owns one pixel.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

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

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// ---------------------------------------------------------------------------
// Descriptors.  grid (ceil(W/blockDim), H, K).
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void lf_descriptors_kernel(const uint8_t *__restrict__ views,
                                                             typename Pair<ST>::T *__restrict__ feat,
                                                             int H, int W) {
    const int k = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const uint8_t *v = views + (size_t)k * H * W * 3;
    int L[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int yy = clampi(y + r - 1, 0, H - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int xx = clampi(x + c - 1, 0, W - 1);
            const uint8_t *px = v + ((size_t)yy * W + xx) * 3;
            L[r][c] = (int)px[0] + (int)px[1] + (int)px[2];
        }
    }
    const int gx = (L[0][2] - L[0][0]) + 2 * (L[1][2] - L[1][0]) + (L[2][2] - L[2][0]);
    const int gy = (L[2][0] - L[0][0]) + 2 * (L[2][1] - L[0][1]) + (L[2][2] - L[0][2]);
    const float s = 1.0f / 4096.0f;  // exact: |G| <= 3060
    feat[((size_t)k * H + y) * W + x] = make_pair<ST>((float)gx * s, (float)gy * s);
}

// ---------------------------------------------------------------------------
// Ray prior and first weights.  grid (ceil(W/blockDim), H, K).
// ---------------------------------------------------------------------------
struct PriorArgs {
    const float *S_P, *mu_T, *q_warm;
    float *rho, *q;
    uint32_t *bad;  // count of invalid input values (device-resident inputs only)
    int K, H, W, storage, check;
    float tau;
    float b[kMaxViews];
};

__global__ __launch_bounds__(256) void lf_ray_prior_kernel(PriorArgs a) {
    const int k = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.W) return;
    const size_t pix = (size_t)y * a.W + x;
    const size_t i = (size_t)k * a.H * a.W + pix;
    const float mu = a.mu_T[pix];
    const float *row = a.S_P + ((size_t)k * a.H + y) * a.W;
    int i0;
    float t;
    footprint(x, a.b[k], mu, i0, t);
    const float s0 = as_stored(row[clampi(i0, 0, a.W - 1)], a.storage);
    const float s1 = as_stored(row[clampi(i0 + 1, 0, a.W - 1)], a.storage);
    const float r = lerp(s0, s1, t);
    a.rho[i] = r;
    float q0 = (r >= a.tau) ? 1.0f : 0.0f;
    if (a.q_warm) q0 = a.q_warm[i];
    a.q[i] = q0;
    if (a.check) {
        const float s = row[x];
        uint32_t nbad = !(s >= 0.0f && s <= 1.0f);
        if (k == 0) nbad += !(fabsf(mu) <= 1e6f);
        if (a.q_warm) nbad += !(q0 >= 0.0f && q0 <= 1.0f);
        if (nbad) atomicAdd(a.bad, nbad);
    }
}

// ---------------------------------------------------------------------------
// EM iterations.  grid (ceil(W/tile), H), block = tile threads, one pixel per
// lane.  Dynamic LDS: the descriptor window of every view for this tile.
// ---------------------------------------------------------------------------
struct EmArgs {
    const void *feat;     // [K][H][W] pairs at storage precision
    const float *rho;     // [K][H][W]
    const float *mu_T;    // [H][W]
    float *q;             // [K][H][W], read at entry, written at exit
    int32_t *d_idx;       // [H][W]
    float *lpix;          // [H][W], objective of the last iteration
    double *obj;          // [n_iters][n_blocks] block sums of the objective
    int H, W, D, n_iters, n_blocks, tile, mode;
    int dmin_i, dstep_i;  // integer levels (integer-shift path)
    float d_min, d_step;
    float beta_p;         // beta / K
    float lambda, gamma;
    float c_exp2;         // log2(e) / (2 sigma^2)
    float c_exp;          // 1 / (2 sigma^2)
    int bi[kMaxViews];    // integer baselines (integer-shift path)
    float b[kMaxViews];
};

struct Window {
    int umin, off, len;  // first staged position, offset in LDS (pairs), staged length
};

template <int K, bool FRAC>
__device__ __forceinline__ void view_windows(const EmArgs &a, int x0, Window (&w)[K], int &total) {
    int off = 0;
    const float d_max = a.d_min + (float)(a.D - 1) * a.d_step;
    const int dmax_i = a.dmin_i + (a.D - 1) * a.dstep_i;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int umin, umax;
        if (FRAC) {
            const float s0 = a.b[k] * a.d_min, s1 = a.b[k] * d_max;
            umin = (int)floorf((float)x0 - fmaxf(s0, s1)) - 2;
            umax = (int)floorf((float)(x0 + a.tile - 1) - fminf(s0, s1)) + 3;
        } else {
            const int s0 = a.bi[k] * a.dmin_i, s1 = a.bi[k] * dmax_i;
            umin = x0 - max(s0, s1);
            umax = x0 + a.tile - 1 - min(s0, s1);
        }
        w[k].umin = umin;
        w[k].off = off;
        w[k].len = umax - umin + 1;
        off += w[k].len;
    }
    total = off;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <int K, int ST, bool FRAC>
__device__ __forceinline__ void gather(const typename Pair<ST>::T *win, const Window (&w)[K], const EmArgs &a,
                                       int x, int j, float2 (&f)[K]) {
    if (FRAC) {
        const float d = fmaf((float)j, a.d_step, a.d_min);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int i0;
            float t;
            footprint(x, a.b[k], d, i0, t);
            // the window margins cover float rounding of the footprint; the
            // clamp keeps every read inside this view's window regardless
            const int p = clampi(w[k].off + i0 - w[k].umin, w[k].off, w[k].off + w[k].len - 2);
            const float2 v0 = widen(win[p]), v1 = widen(win[p + 1]);
            f[k] = make_float2(lerp(v0.x, v1.x, t), lerp(v0.y, v1.y, t));
        }
    } else {
        const int d = a.dmin_i + j * a.dstep_i;
#pragma unroll
        for (int k = 0; k < K; ++k) f[k] = widen(win[w[k].off + x - a.bi[k] * d - w[k].umin]);
    }
}

template <int K, int ST, bool FRAC>
__global__ __launch_bounds__(256) void lf_em_kernel(EmArgs a) {
    using P = typename Pair<ST>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    P *win = reinterpret_cast<P *>(lds_raw);
    __shared__ double red[8];

    const int y = blockIdx.y;
    const int x0 = blockIdx.x * a.tile;
    const int tid = threadIdx.x;
    const int x = x0 + tid;
    const bool active = x < a.W;
    const size_t HW = (size_t)a.H * a.W;
    const size_t pix = (size_t)y * a.W + x;

    Window w[K];
    int total;
    view_windows<K, FRAC>(a, x0, w, total);

    // Stage the windows (replicated border outside the image).
    const P *feat = reinterpret_cast<const P *>(a.feat);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const P *row = feat + ((size_t)k * a.H + y) * a.W;
        for (int p = tid; p < w[k].len; p += blockDim.x) win[w[k].off + p] = row[clampi(w[k].umin + p, 0, a.W - 1)];
    }
    __syncthreads();

    float q[K], la[K], lb[K];
    float mu = 0.0f;
    if (active) {
        mu = a.mu_T[pix];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float r = a.rho[k * HW + pix];
            q[k] = a.q[k * HW + pix];
            la[k] = (r > 0.0f ? logf(r) : -INFINITY) + a.lambda;   // ln rho + lambda
            lb[k] = (r < 1.0f ? log1pf(-r) : -INFINITY);           // ln(1 - rho)
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) q[k] = la[k] = lb[k] = 0.0f;
    }

    int best_j = 0;
    float L = 0.0f;
    const int block_id = blockIdx.y * gridDim.x + blockIdx.x;
    for (int it = 0; it < a.n_iters; ++it) {
        if (active) {
            // ---- M-step: weights from the previous E-step (or the start) ----
            float Q = 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) Q += q[k];
            const bool empty = !(Q > 0.0f);
            float wt[K];
#pragma unroll
            for (int k = 0; k < K; ++k) wt[k] = empty ? 1.0f : q[k];
            const float invW = 1.0f / (empty ? (float)K : Q);
            const float cw = empty ? 0.0f : a.beta_p;
            float best_E = INFINITY;
            best_j = 0;
            for (int j = 0; j < a.D; ++j) {
                float2 f[K];
                gather<K, ST, FRAC>(win, w, a, x, j, f);
                float mx = 0.0f, my = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    mx = fmaf(wt[k], f[k].x, mx);
                    my = fmaf(wt[k], f[k].y, my);
                }
                mx *= invW;
                my *= invW;
                float C = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float dx = f[k].x - mx, dy = f[k].y - my;
                    C = fmaf(wt[k], fmaf(dx, dx, dy * dy), C);
                }
                const float t = fmaf((float)j, a.d_step, a.d_min) - mu;
                const float g = __builtin_amdgcn_exp2f(-(t * t) * a.c_exp2);
                const float E = fmaf(cw, C, -kLn2 * __builtin_amdgcn_logf(a.gamma + g));
                if (E < best_E) {
                    best_E = E;
                    best_j = j;
                }
            }
            // ---- E-step at the new disparity ----
            float2 f[K];
            gather<K, ST, FRAC>(win, w, a, x, best_j, f);
            float mx = 0.0f, my = 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                mx = fmaf(wt[k], f[k].x, mx);
                my = fmaf(wt[k], f[k].y, my);
            }
            mx *= invW;
            my *= invW;
            const float t = fmaf((float)best_j, a.d_step, a.d_min) - mu;
            L = logf(a.gamma + expf(-(t * t) * a.c_exp));
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float dx = f[k].x - mx, dy = f[k].y - my;
                const float e = fmaf(dx, dx, dy * dy);
                const float a1 = la[k] - a.beta_p * e;
                const float a0 = lb[k];
                if (a.mode == 1) {
                    q[k] = (a1 >= a0) ? 1.0f : 0.0f;
                    L += fmaxf(a1, a0);
                } else {
                    q[k] = 1.0f / (1.0f + __expf(a0 - a1));
                    const float hi = fmaxf(a1, a0);
                    L += hi + log1pf(expf(-fabsf(a1 - a0)));
                }
            }
        }
        // ---- FP64 block sum of the objective ----
        double s = wave_sum(active ? (double)L : 0.0);
        const int lane = tid & 63, wv = tid >> 6;
        if (lane == 0) red[wv] = s;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) tot += red[i];
            a.obj[(size_t)it * a.n_blocks + block_id] = tot;
        }
        __syncthreads();
    }
    if (active && a.n_iters > 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) a.q[k * HW + pix] = q[k];
        a.d_idx[pix] = best_j;
        a.lpix[pix] = L;
    }
}

// ---------------------------------------------------------------------------
// Refocus (Eq. 2).  grid (ceil(W/blockDim), H).
// ---------------------------------------------------------------------------
struct RefocusArgs {
    const uint8_t *views;
    const int32_t *d_idx;
    const float *q;
    float *rgb;
    uint8_t *hole;
    int K, H, W, ref, frac;
    int dmin_i, dstep_i;
    float d_min, d_step;
    int bi[kMaxViews];
    float b[kMaxViews];
};

__global__ __launch_bounds__(256) void lf_refocus_kernel(RefocusArgs a) {
    const int y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.W) return;
    const size_t HW = (size_t)a.H * a.W;
    const size_t pix = (size_t)y * a.W + x;
    const int j = a.d_idx[pix];
    float acc[3] = {0.0f, 0.0f, 0.0f};
    int n = 0;
    if (!a.frac) {
        int iacc[3] = {0, 0, 0};
        const int d = a.dmin_i + j * a.dstep_i;
        for (int k = 0; k < a.K; ++k) {
            if (!(a.q[k * HW + pix] >= 0.5f)) continue;
            const int u = clampi(x - a.bi[k] * d, 0, a.W - 1);
            const uint8_t *px = a.views + (((size_t)k * a.H + y) * a.W + u) * 3;
            iacc[0] += px[0];
            iacc[1] += px[1];
            iacc[2] += px[2];
            ++n;
        }
        acc[0] = (float)iacc[0];
        acc[1] = (float)iacc[1];
        acc[2] = (float)iacc[2];
    } else {
        const float d = fmaf((float)j, a.d_step, a.d_min);
        for (int k = 0; k < a.K; ++k) {
            if (!(a.q[k * HW + pix] >= 0.5f)) continue;
            int i0;
            float t;
            footprint(x, a.b[k], d, i0, t);
            const uint8_t *r = a.views + ((size_t)k * a.H + y) * a.W * 3;
            const uint8_t *p0 = r + (size_t)clampi(i0, 0, a.W - 1) * 3;
            const uint8_t *p1 = r + (size_t)clampi(i0 + 1, 0, a.W - 1) * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += lerp((float)p0[c], (float)p1[c], t);
            ++n;
        }
    }
    float *o = a.rgb + pix * 3;
    if (n > 0) {
        const float den = 255.0f * (float)n;
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = acc[c] / den;
        if (a.hole) a.hole[pix] = 0;
    } else {
        const uint8_t *c_ref = a.views + (((size_t)a.ref * a.H + y) * a.W + x) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = (float)c_ref[c] / 255.0f;
        if (a.hole) a.hole[pix] = 1;
    }
}

// ---------------------------------------------------------------------------
// 3x3 per-channel median with replicated border.  grid (ceil(W/blockDim), H).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cswap(float &p, float &q) {
    const float lo = fminf(p, q), hi = fmaxf(p, q);
    p = lo;
    q = hi;
}

__global__ __launch_bounds__(256) void lf_median3_kernel(const float *__restrict__ in, float *__restrict__ out,
                                                         int H, int W) {
    const int y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int s = 0; s < 3; ++s)
                v[r * 3 + s] = in[((size_t)clampi(y + r - 1, 0, H - 1) * W + clampi(x + s - 1, 0, W - 1)) * 3 + c];
        // median of 9 by a full sorting network on the nine values
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int m = (i & 1); m + 1 < 9; m += 2) cswap(v[m], v[m + 1]);
        out[((size_t)y * W + x) * 3 + c] = v[4];
    }
}

}  // namespace lfem
