// Host side of the C ABI declared in include/lf_em.h: parameter validation,
// device buffer plan, precision and view-count dispatch, launches and copies.
#include "lf_em.h"
#include "lf_frame_kernels.h"
#include "lf_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace lfem {

thread_local std::string g_last_error;

lf_status set_error(lf_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

lf_status hip_error(hipError_t e, const char *what) {
    return set_error(LF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define LF_HIP(call, what)                                 \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_error(e_, what);  \
    } while (0)

static bool is_int(float v) { return std::isfinite(v) && std::fabs(v) < (1 << 20) && std::floor(v) == v; }

lf_status validate_params(const lf_params *p) {
    if (!p) return set_error(LF_EINVAL, "params is NULL");
    if (p->K < 2 || p->K > LF_MAX_VIEWS) return set_error(LF_EINVAL, "K=%d outside [2,%d]", p->K, LF_MAX_VIEWS);
    if (p->H < 1 || p->W < 1) return set_error(LF_EINVAL, "H=%d W=%d must be >= 1", p->H, p->W);
    if ((int64_t)p->H * p->W > (int64_t)1 << 28) return set_error(LF_EINVAL, "frame too large");
    if (p->ref < 0 || p->ref >= p->K) return set_error(LF_EINVAL, "ref=%d outside [0,K)", p->ref);
    for (int k = 0; k < p->K; ++k)
        if (!std::isfinite(p->baselines[k]) || std::fabs(p->baselines[k]) > 1e4f)
            return set_error(LF_EINVAL, "baselines[%d] not finite or too large", k);
    if (p->baselines[p->ref] != 0.0f) return set_error(LF_EINVAL, "baselines[ref] must be 0");
    if (p->D < 1) return set_error(LF_EINVAL, "D=%d must be >= 1", p->D);
    if (!(p->d_step > 0.0f) || !std::isfinite(p->d_step)) return set_error(LF_EINVAL, "d_step must be > 0");
    if (!std::isfinite(p->d_min)) return set_error(LF_EINVAL, "d_min not finite");
    if (!std::isfinite(p->d_min + (p->D - 1) * p->d_step) || std::fabs(p->d_min + (p->D - 1) * p->d_step) > 1e5f)
        return set_error(LF_EINVAL, "disparity range too large");
    {
        // footprints x - b_k d are formed in float: keep |b_k d| where a float
        // resolves well below one pixel
        float bmax = 0.0f;
        for (int k = 0; k < p->K; ++k) bmax = std::max(bmax, std::fabs(p->baselines[k]));
        const float dabs = std::max(std::fabs(p->d_min), std::fabs(p->d_min + (p->D - 1) * p->d_step));
        if ((double)bmax * dabs > 1e6) return set_error(LF_EINVAL, "shift |baseline * disparity| above 1e6 pixels");
    }
    if (!(p->beta >= 0.0f) || !std::isfinite(p->beta)) return set_error(LF_EINVAL, "beta must be finite and >= 0");
    if (std::isnan(p->lambda) && !(p->beta > 0.0f))
        return set_error(LF_EINVAL, "lambda cannot be derived for beta == 0; pass it explicitly");
    if (!std::isnan(p->lambda) && !std::isfinite(p->lambda)) return set_error(LF_EINVAL, "lambda must be finite or NaN");
    if (!(p->gamma > 0.0f) || !std::isfinite(p->gamma)) return set_error(LF_EINVAL, "gamma must be > 0");
    if (!(p->sigma > 0.0f) || !std::isfinite(p->sigma)) return set_error(LF_EINVAL, "sigma must be > 0");
    if (!(p->tau_init >= 0.0f && p->tau_init <= 1.0f)) return set_error(LF_EINVAL, "tau_init outside [0,1]");
    if (p->storage < LF_F32 || p->storage > LF_BF16) return set_error(LF_EINVAL, "storage=%d unknown", p->storage);
    if (p->mode < LF_SOFT || p->mode > LF_ENUM_HARD) return set_error(LF_EINVAL, "mode=%d unknown", p->mode);
    if (p->mode >= LF_ENUM_SOFT && p->K > LF_ENUM_MAX_VIEWS)
        return set_error(LF_EINVAL, "K=%d above %d in an enumeration mode", p->K, LF_ENUM_MAX_VIEWS);
    if (p->flags & ~(LF_INPUTS_ON_DEVICE | LF_OUTPUTS_ON_DEVICE | LF_EXHAUSTIVE_SWEEP | LF_PRIOR_WINDOW |
                     LF_DYNAMIC_ONLY | LF_DEFERRED_CHECK))
        return set_error(LF_EINVAL, "unknown flags");
    return LF_OK;
}

lf_status validate_host_values(const lf_params *p, const float *S_P, const float *mu_T, const float *q_warm) {
    const size_t HW = (size_t)p->H * p->W, KHW = HW * p->K;
    for (size_t i = 0; i < KHW; ++i)
        if (!(S_P[i] >= 0.0f && S_P[i] <= 1.0f)) return set_error(LF_EINVAL, "S_P[%zu] outside [0,1] or NaN", i);
    for (size_t i = 0; i < HW; ++i)
        if (!(std::fabs(mu_T[i]) <= 1e6f)) return set_error(LF_EINVAL, "mu_T[%zu] not finite or above 1e6", i);
    if (q_warm)
        for (size_t i = 0; i < KHW; ++i)
            if (!(q_warm[i] >= 0.0f && q_warm[i] <= 1.0f)) return set_error(LF_EINVAL, "q_warm[%zu] outside [0,1]", i);
    return LF_OK;
}

float derived_lambda(const lf_params *p) {
    if (!std::isnan(p->lambda)) return p->lambda;
    const double F = 2.0, bp = (double)p->beta / p->K, R = 3060.0 / 4096.0, pi = 3.14159265358979323846;
    return (float)(0.5 * F * std::log(bp / pi) + F * std::log(2.0 * R));
}

Geometry make_geometry(const lf_params *p) {
    Geometry g{};
    g.frac = !(is_int(p->d_min) && is_int(p->d_step));
    for (int k = 0; k < p->K; ++k) {
        if (!is_int(p->baselines[k])) g.frac = true;
        g.bi[k] = g.frac ? 0 : (int)p->baselines[k];
    }
    g.dmin_i = g.frac ? 0 : (int)p->d_min;
    g.dstep_i = g.frac ? 0 : (int)p->d_step;
    g.sym = !g.frac && g.dstep_i == 1 && p->ref == (p->K - 1) / 2;
    for (int k = 0; k < p->K && g.sym; ++k)
        if (g.bi[k] != k - p->ref) g.sym = false;
    if (!g.frac) {
        // integer levels must also keep integer shifts inside int range
        for (int k = 0; k < p->K; ++k) {
            const long long s = (long long)std::abs(g.bi[k]) *
                                (std::llabs((long long)g.dmin_i) + (long long)(p->D - 1) * g.dstep_i);
            if (s > (1 << 24)) g.frac = true;
        }
    }
    return g;
}

// Upper bound of the LDS pairs one EM block stages for a tile of `tile` pixels.
size_t em_window_pairs(const lf_params *p, const Geometry &g, int tile) {
    size_t tot = 0;
    const double d_max = (double)p->d_min + (double)(p->D - 1) * p->d_step;
    for (int k = 0; k < p->K; ++k) {
        if (g.frac) {
            const double s0 = (double)p->baselines[k] * p->d_min, s1 = (double)p->baselines[k] * d_max;
            tot += (size_t)tile + (size_t)std::ceil(std::fabs(s1 - s0)) + 8;
        } else {
            const long long dmax_i = g.dmin_i + (long long)(p->D - 1) * g.dstep_i;
            const long long s0 = (long long)g.bi[k] * g.dmin_i, s1 = (long long)g.bi[k] * dmax_i;
            const size_t len = (size_t)tile + (size_t)std::llabs(s1 - s0);
            tot += len;
        }
    }
    return tot;
}

// Positions of the widest single view window of a tile of `tile` pixels.
size_t em_window_widest(const lf_params *p, const Geometry &g, int tile) {
    size_t widest = 0;
    for (int k = 0; k < p->K; ++k) {
        lf_params one = *p;
        one.K = 1;
        one.baselines[0] = p->baselines[k];
        Geometry g1 = g;
        g1.bi[0] = g.bi[k];
        widest = std::max(widest, em_window_pairs(&one, g1, tile));
    }
    return widest;
}

size_t pair_bytes(int storage) { return storage == LF_F32 ? 8 : 4; }

// LDS record of one staged position in the EM kernel: the pair plus |f|^2,
// 8 bytes for every storage format (FP32 descriptors as binary16 or int16).
size_t rec_bytes(int storage) { (void)storage; return 8; }

// ---------------------------------------------------------------------------
// Kernel dispatch over (K, storage, integer/fractional shifts, sweep kind).
// ---------------------------------------------------------------------------
// The fast sweep shares levels across a wave's lanes unless a search window
// is set (its short ranges gain too little to pay for the prior bound).
EmKernel pick_em(const lf_params *p, const Geometry &g) {
    const bool exh = (p->flags & LF_EXHAUSTIVE_SWEEP) != 0, share = !(p->flags & LF_PRIOR_WINDOW);
    const bool enumerate = p->mode == LF_ENUM_SOFT || p->mode == LF_ENUM_HARD;
    switch (p->storage) {
        case LF_F32: return pick_em_f32(p->K, g.frac, exh, g.sym, share, enumerate);
        case LF_F16: return pick_em_f16(p->K, g.frac, exh, g.sym, share, enumerate);
        default: return pick_em_bf16(p->K, g.frac, exh, g.sym, share, enumerate);
    }
}

// ---------------------------------------------------------------------------
// Launch helpers shared by the plain context and the server.
// ---------------------------------------------------------------------------
// The load pass (descriptors and ray prior, one launch).
hipError_t launch_load(const lf_params *p, const uint8_t *views, void *feat, const float *S_P, const float *mu_T,
                       const float *q_warm, float *rho, float *omr, float *q, uint32_t *bad, int check,
                       hipStream_t s) {
    PriorArgs a{};
    a.S_P = S_P;
    a.mu_T = mu_T;
    a.q_warm = q_warm;
    a.rho = rho;
    a.omr = omr;
    a.q = q;
    a.bad = bad;
    a.K = p->K;
    a.H = p->H;
    a.W = p->W;
    a.storage = p->storage;
    a.check = check;
    a.tau = p->tau_init;
    for (int k = 0; k < p->K; ++k) a.b[k] = p->baselines[k];
    dim3 block(256), grid((p->W + 255) / 256, (p->H + kDescRows - 1) / kDescRows + p->H, p->K);
    switch (p->storage) {
        case LF_F32:
            hipLaunchKernelGGL(lf_load_kernel<0>, grid, block, 0, s, views, (float2 *)feat, a);
            break;
        case LF_F16:
            hipLaunchKernelGGL(lf_load_kernel<1>, grid, block, 0, s, views, (__half2 *)feat, a);
            break;
        default:
            hipLaunchKernelGGL(lf_load_kernel<2>, grid, block, 0, s, views, (uint32_t *)feat, a);
            break;
    }
    return hipGetLastError();
}

// Dynamic-only work list: items of up to 64 dynamic reference pixels of a
// row within `span` columns (the widest of 256, 192, 128, 64 whose view
// windows fit a block's LDS), one wave each; with the shared sweep (integer
// shifts, no search window, not the exhaustive sweep) also of at most
// kItemUnbounded pixels predicted unbounded, within a budget of W/64 such
// cuts per row.
DynPlan dyn_plan(const lf_params *p, const Geometry &g, size_t lds_limit) {
    DynPlan d{};
    if (!(p->flags & LF_DYNAMIC_ONLY)) return d;
    for (int w = 256; w >= 64; w -= 64) {
        d.span = w;
        d.lds = em_window_pairs(p, g, w) * rec_bytes(p->storage);
        if (d.lds <= lds_limit) break;
    }
    d.split = !g.frac && !(p->flags & (LF_EXHAUSTIVE_SWEEP | LF_PRIOR_WINDOW));
    d.per_row = p->W / 64 + p->W / d.span + 1 + (d.split ? p->W / 64 : 0);
    d.max_items = p->H * d.per_row;
    return d;
}

size_t dyn_rows_ints(const lf_params *p, const DynPlan &d) { return (size_t)p->H * (2 * (size_t)d.per_row + 1); }

hipError_t launch_dyn_list(const lf_params *p, const EmArgs &a, const DynPlan &d, int *rows, int4 *items,
                           int *n_items, hipStream_t s) {
    int *counts = rows, *row_items = rows + p->H;
    hipLaunchKernelGGL(lf_dyn_rows_kernel, dim3(p->H), dim3(64), 0, s, a, d.per_row, p->K, p->storage, d.split,
                       counts, row_items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lf_dyn_items_kernel, dim3(1), dim3(256), 0, s, counts, row_items, p->H, d.per_row, items,
                       n_items);
    return hipGetLastError();
}


EmArgs make_em_args(const lf_params *p, const Geometry &g, float lambda) {
    EmArgs a{};
    // kernel view order: the reference first, then the others in array order
    int n = 0;
    a.perm[n++] = p->ref;
    for (int k = 0; k < p->K; ++k)
        if (k != p->ref) a.perm[n++] = k;
    for (int k = 0; k < p->K; ++k) {
        a.bi[k] = g.bi[a.perm[k]];
        a.b[k] = p->baselines[a.perm[k]];
    }
    // |d - mu| beyond which exp(-(d-mu)^2/(2 sigma^2)) < gamma * 2^-28, so that
    // gamma + g rounds to gamma in FP32 (half an ulp of gamma is >= gamma 2^-25)
    {
        const double c2 = 1.4426950408889634 / (2.0 * (double)p->sigma * p->sigma);
        const double e = 28.0 - std::log2((double)p->gamma);
        a.prior_T = e > 0.0 ? (float)std::sqrt(e / c2) : -1.0f;
        // ln(gamma + g) <= ln(1 + gamma) for g <= 1; the slack covers the
        // rounding of gamma + g and the hardware logarithm
        const double hi = std::log1p((double)p->gamma);
        a.prior_hi = (float)(hi + 1e-5 * std::max(1.0, std::fabs(hi)));
    }
    // bound of |one-pass energy - two-pass energy| in FP32 (see the kernel):
    // beta' * (16K + 64) u * S + 64 u (|ln gamma| + 1), u = 2^-24
    {
        const double u = std::ldexp(1.0, -24);
        a.margin_k = (float)((16.0 * p->K + 64.0) * u);
        a.margin_c = (float)(64.0 * u * (std::max(std::fabs(std::log((double)p->gamma)),
                                                  std::log1p((double)p->gamma)) + 1.0));
    }
    a.H = p->H;
    a.W = p->W;
    a.D = p->D;
    a.mode = p->mode;
    a.dmin_i = g.dmin_i;
    a.dstep_i = g.dstep_i;
    a.d_min = p->d_min;
    a.d_step = p->d_step;
    a.beta_p = (float)((double)p->beta / p->K);
    a.beta = p->beta;
    a.lambda = lambda;
    a.gamma = p->gamma;
    const double s2 = 2.0 * (double)p->sigma * p->sigma;
    a.c_exp2 = (float)(1.4426950408889634 / s2);
    a.c_exp = (float)(1.0 / s2);
    a.win_half = (p->flags & LF_PRIOR_WINDOW) ? 3.0f * p->sigma : 0.0f;
    a.dyn_only = (p->flags & LF_DYNAMIC_ONLY) ? 1 : 0;
    a.tau = p->tau_init;
    a.d_absmax = (float)std::max(std::fabs((double)p->d_min),
                                 std::fabs((double)p->d_min + (double)(p->D - 1) * p->d_step));
    a.inv_step = (float)(1.0 / (double)p->d_step);
    a.c_t2 = (float)(s2 * 0.69314718055994530942);
    return a;
}

// Row tiles (grid (ceil(W/tile), H)), or with a dynamic-only work list one
// wave per item (grid d.max_items rounded up to a multiple of 8; blocks past
// the list's length exit).
hipError_t launch_em(const lf_params *p, const Geometry &g, EmArgs a, int tile, size_t lds, hipStream_t s,
                     const DynPlan *d) {
    EmKernel kern = pick_em(p, g);
    a.tile = tile;
    dim3 block(tile), grid((p->W + tile - 1) / tile, p->H);
    a.n_blocks = grid.x * grid.y;
    if (a.items) {
        // one wave per item; the objective has a slot per possible item, and
        // the grid is rounded up to a multiple of 8 (the items are dealt to
        // the XCDs in groups)
        a.seg_w = d->span;
        block = dim3(64);
        grid = dim3((d->max_items + 7) & ~7);
        a.n_blocks = d->max_items;
        lds = d->lds;
    }
    hipLaunchKernelGGL(kern, grid, block, lds, s, a);
    return hipGetLastError();
}

RefocusArgs make_refocus_args(const lf_params *p, const Geometry &g) {
    RefocusArgs r{};
    r.K = p->K;
    r.H = p->H;
    r.W = p->W;
    r.ref = p->ref;
    r.frac = g.frac;
    r.dmin_i = g.dmin_i;
    r.dstep_i = g.dstep_i;
    r.d_min = p->d_min;
    r.d_step = p->d_step;
    for (int k = 0; k < p->K; ++k) {
        r.bi[k] = g.bi[k];
        r.b[k] = p->baselines[k];
    }
    return r;
}

hipError_t launch_refocus(const lf_params *p, RefocusArgs r, hipStream_t s) {
    dim3 block(256), grid((p->W + 255) / 256, p->H);
    hipLaunchKernelGGL(lf_refocus_kernel, grid, block, 0, s, r);
    return hipGetLastError();
}

hipError_t launch_median3(const lf_params *p, const float *in, float *out, hipStream_t s) {
    dim3 block(256), grid((p->W + 255) / 256, p->H);
    hipLaunchKernelGGL(lf_median3_kernel, grid, block, 0, s, in, out, p->H, p->W);
    return hipGetLastError();
}

// Refocus of the current state (Eq. 2) into rgb (through rgb_med and the 3x3
// median when median == 3), the holes into hole (nullable); d_out / q_out
// (nullable) receive device copies of the level and weights in the same pass.
hipError_t launch_refocus_frame(const lf_params *p, const Geometry &g, const uint8_t *views, const int32_t *d_idx,
                                const float *q, const float *rho, float *rgb, uint8_t *hole, float *rgb_med,
                                int median, int32_t *d_out, float *q_out, hipStream_t s) {
    RefocusArgs r = make_refocus_args(p, g);
    r.views = views;
    r.d_idx = d_idx;
    r.q = q;
    r.rho_ref = (p->flags & LF_DYNAMIC_ONLY) ? rho + (size_t)p->ref * p->H * p->W : nullptr;
    r.tau = p->tau_init;
    r.rgb = median ? rgb_med : rgb;
    r.hole = hole;
    r.d_out = d_out;
    r.q_out = q_out;
    hipError_t e = launch_refocus(p, r, s);
    if (e == hipSuccess && median) e = launch_median3(p, rgb_med, rgb, s);
    return e;
}

// objective[t] = sum over blocks b, in block order, of partials[t][b] for
// t < n: the same additions in the same order as the host sum of the plain
// context, so both give the same bits.
hipError_t launch_objective_sum(const double *partials, int n_blocks, int n, double *objective, hipStream_t s) {
    hipLaunchKernelGGL(lf_objective_sum_kernel, dim3((n + 63) / 64), dim3(64), 0, s, partials, n_blocks, n, objective);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(lf_fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int32_t *)p, n,
                       (int32_t)v);
    return hipGetLastError();
}

// Row-tile width of the EM kernel: the width (a multiple of the 64-lane
// wave, up to 256) with the best product of waves resident per SIMD (capped
// at 4; bounded by the kernel's VGPRs and the CU's LDS) and lanes doing
// work (W over W rounded up to whole tiles); ties go to the narrower tile.
// Returns 0 when not even 64 columns fit the block LDS limit.
int choose_tile(const lf_params *p, const Geometry &g, size_t lds_limit, size_t lds_per_cu, int vgprs,
                size_t *lds_out) {
    const int waves_simd_vgpr = vgprs > 0 ? 512 / ((vgprs + 7) / 8 * 8) : 4;
    int best = 0;
    double best_score = -1.0;
    *lds_out = em_window_pairs(p, g, 64) * rec_bytes(p->storage);
    for (int tile = 64; tile <= 256; tile += 64) {
        if (tile > 64 && tile - 64 >= p->W) break;   // wider than the frame
        const size_t lds = em_window_pairs(p, g, tile) * rec_bytes(p->storage) + 64;
        if (lds > lds_limit) continue;
        const int wb = tile / 64;
        const int blocks_lds = (int)(lds_per_cu / lds);
        const int blocks_vgpr = 4 * std::max(waves_simd_vgpr, 1) / wb;
        const int blocks = std::min(blocks_lds, blocks_vgpr);
        if (blocks < 1) continue;
        const double per_simd = std::min(blocks * wb / 4.0, 4.0);
        const double used = (double)p->W / (double)(((p->W + tile - 1) / tile) * tile);
        const double score = per_simd * used;
        if (score > best_score + 1e-9) {
            best_score = score;
            best = tile;
            *lds_out = em_window_pairs(p, g, tile) * rec_bytes(p->storage);
        }
    }
    return best;
}

lf_status em_launch_shape(const lf_params *p, const Geometry &g, int device, int *tile, size_t *lds) {
    size_t lds_limit = 0;
    {
        int v = 0;
        hipError_t e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
        if (e != hipSuccess) return hip_error(e, "device attribute");
        lds_limit = (size_t)v;
    }
    size_t lds_cu = 0;
    {
        int v = 0;
        hipError_t e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device);
        if (e != hipSuccess) return hip_error(e, "device attribute");
        lds_cu = v > 0 ? (size_t)v : lds_limit;
    }
    int vgprs = 0;
    {
        // the tile follows the fast sweep's kernel also when the exhaustive
        // sweep is asked for, so that both use the same blocks and the
        // objective's FP64 block sums add up in the same order
        lf_params pf = *p;
        pf.flags &= ~(uint32_t)LF_EXHAUSTIVE_SWEEP;
        EmKernel kern = pick_em(&pf, g);
        hipFuncAttributes fa;
        if (kern && hipFuncGetAttributes(&fa, (const void *)kern) == hipSuccess) vgprs = fa.numRegs;
        (void)hipGetLastError();
    }
    *tile = choose_tile(p, g, lds_limit, lds_cu, vgprs, lds);
    if (!*tile)
        return set_error(LF_EINVAL, "disparity halo needs %zu bytes of LDS per block, more than %zu", *lds, lds_limit);
    return LF_OK;
}

}  // namespace lfem

using namespace lfem;

// ---------------------------------------------------------------------------
// Plain context.
// ---------------------------------------------------------------------------
struct lf_ctx {
    lf_params p;
    Geometry g;
    float lambda;
    int device;
    hipStream_t stream;
    bool own_stream;
    DeviceArena arena;
    uint8_t *views_own;
    float *sp_own, *mu_own, *qw_own;
    const uint8_t *views;   // the frame's views on the device (own copy or caller's)
    const float *mu_dev;    // the frame's mu_T on the device (own copy or caller's)
    void *feat;
    float *rho, *omr, *q, *lpix, *rgb, *rgb_med;
    int32_t *d_idx;
    int32_t *seg_keys;      // per-view segmentation: ray seen at each view pixel
    uint8_t *seg_labels;    // per-view segmentation labels (host-output staging)
    uint8_t *hole;
    double *obj;
    uint32_t *bad;
    unsigned long long *sweep;  // level-step counter of lf_em_sweep_count
    DynPlan dyn;            // dynamic-only work list (span 0: none)
    int *dyn_rows;          // [H] items per row, then [H][per_row] their first columns
    int4 *dyn_items;        // [max_items] (row, first column, pixels, 0)
    int *dyn_n;             // number of items
    double *h_obj;          // pinned
    uint32_t *h_bad;        // pinned
    bool check_pending;     // deferred value check of device inputs not yet read
    int tile, n_blocks;
    size_t lds;
    bool loaded;
    int64_t iters;
};



static lf_status ctx_alloc(lf_ctx *c) {
    const lf_params &p = c->p;
    const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
    const bool dev_in = p.flags & LF_INPUTS_ON_DEVICE;
    const bool dev_out = p.flags & LF_OUTPUTS_ON_DEVICE;
    lf_status st0 = em_launch_shape(&p, c->g, c->device, &c->tile, &c->lds);
    if (st0 != LF_OK) return st0;
    c->n_blocks = ((p.W + c->tile - 1) / c->tile) * p.H;
    {
        int v = 0;
        LF_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device), "device attribute");
        c->dyn = dyn_plan(&p, c->g, (size_t)v);
        if (c->dyn.span) c->n_blocks = c->dyn.max_items;
    }
    ArenaPlan plan;
    if (!dev_in) {
        plan.add(&c->views_own, KHW * 3);
        plan.add(&c->sp_own, KHW * 4);
        plan.add(&c->mu_own, HW * 4);
        plan.add(&c->qw_own, KHW * 4);
    }
    plan.add(&c->feat, KHW * pair_bytes(p.storage));
    plan.add(&c->rho, KHW * 4);
    plan.add(&c->omr, KHW * 4);
    plan.add(&c->q, KHW * 4);
    plan.add(&c->d_idx, HW * 4);
    plan.add(&c->lpix, HW * 4);
    plan.add(&c->obj, (size_t)kMaxItersPerLaunch * c->n_blocks * 8);
    plan.add(&c->bad, 256);
    plan.add(&c->sweep, 256);
    if (c->dyn.span) {
        plan.add(&c->dyn_rows, dyn_rows_ints(&p, c->dyn) * 4);
        plan.add(&c->dyn_items, (size_t)c->dyn.max_items * 16);
        plan.add(&c->dyn_n, 256);
    }
    if (!dev_out) {
        plan.add(&c->rgb, HW * 12);
        plan.add(&c->hole, HW);
    }
    plan.add(&c->rgb_med, HW * 12);
    plan.add(&c->seg_keys, KHW * 4);
    if (!dev_out) plan.add(&c->seg_labels, KHW);
    lf_status st = c->arena.allocate(plan);
    if (st != LF_OK) return st;
    LF_HIP(hipHostMalloc((void **)&c->h_obj, (size_t)kMaxItersPerLaunch * c->n_blocks * 8, hipHostMallocDefault),
           "pinned allocation");
    LF_HIP(hipHostMalloc((void **)&c->h_bad, 256, hipHostMallocDefault), "pinned allocation");
    return LF_OK;
}

static lf_status ctx_load(lf_ctx *c, const uint8_t *views, const float *S_P, const float *mu_T, const float *q_warm) {
    const lf_params &p = c->p;
    const size_t HW = (size_t)p.H * p.W, KHW = HW * p.K;
    if (!views || !S_P || !mu_T) return set_error(LF_EINVAL, "views, S_P and mu_T are required");
    const bool dev_in = p.flags & LF_INPUTS_ON_DEVICE;
    c->loaded = false;
    c->iters = 0;
    const float *sp = S_P, *mu = mu_T, *qw = q_warm;
    if (!dev_in) {
        lf_status st = validate_host_values(&p, S_P, mu_T, q_warm);
        if (st != LF_OK) return st;
        LF_HIP(hipMemcpyAsync(c->views_own, views, KHW * 3, hipMemcpyHostToDevice, c->stream), "copy views");
        LF_HIP(hipMemcpyAsync(c->sp_own, S_P, KHW * 4, hipMemcpyHostToDevice, c->stream), "copy S_P");
        LF_HIP(hipMemcpyAsync(c->mu_own, mu_T, HW * 4, hipMemcpyHostToDevice, c->stream), "copy mu_T");
        if (q_warm) LF_HIP(hipMemcpyAsync(c->qw_own, q_warm, KHW * 4, hipMemcpyHostToDevice, c->stream), "copy q_warm");
        c->views = c->views_own;
        sp = c->sp_own;
        mu = c->mu_own;
        qw = q_warm ? c->qw_own : nullptr;
    } else {
        c->views = views;
        // with a deferred check the counter stays set until it is reported
        if (!(p.flags & LF_DEFERRED_CHECK)) LF_HIP(hipMemsetAsync(c->bad, 0, 4, c->stream), "clear counter");
    }
    LF_HIP(launch_load(&p, c->views, c->feat, sp, mu, qw, c->rho, c->omr, c->q, c->bad, dev_in ? 1 : 0, c->stream),
           "load launch");
    if (c->dyn.span) {
        EmArgs da = make_em_args(&p, c->g, c->lambda);
        da.feat = c->feat;
        da.rho = c->rho;
        da.q = c->q;
        da.mu_T = mu;
        da.d_idx = c->d_idx;
        da.lpix = c->lpix;
        da.seg_w = c->dyn.span;
        LF_HIP(launch_dyn_list(&p, da, c->dyn, c->dyn_rows, c->dyn_items, c->dyn_n, c->stream),
               "dynamic-only work list");
    }
    if (dev_in) {
        if (p.flags & LF_DEFERRED_CHECK) {
            // the counter is read by the next call that waits for the stream;
            // no copy per frame
            c->check_pending = true;
        } else {
            LF_HIP(hipMemcpyAsync(c->h_bad, c->bad, 4, hipMemcpyDeviceToHost, c->stream), "copy counter");
            LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
            if (*c->h_bad) return set_error(LF_EINVAL, "%u input values invalid (S_P outside [0,1], mu_T not finite "
                                                      "or q_warm outside [0,1])", *c->h_bad);
        }
    } else {
        // host inputs were copied asynchronously from caller memory: finish the
        // copies before returning so the caller may free its buffers
        LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
    }
    c->mu_dev = mu;
    c->loaded = true;
    return LF_OK;
}

namespace lfem {

lf_status DeviceArena::allocate(const ArenaPlan &plan) {
    release();
    bytes = plan.total();
    if (bytes == 0) return LF_OK;
    hipError_t e = hipMalloc(&base, bytes);
    if (e != hipSuccess) {
        base = nullptr;
        (void)hipGetLastError();
        return set_error(LF_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    size_t off = 0;
    for (const ArenaPlan::Item &i : plan.items) {
        *i.slot = static_cast<char *>(base) + off;
        off += (i.bytes + 255) & ~(size_t)255;
    }
    return LF_OK;
}

void DeviceArena::release() {
    if (base) (void)hipFree(base);
    base = nullptr;
    bytes = 0;
}

}  // namespace lfem

static void ctx_free(lf_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    c->arena.release();
    if (c->h_obj) (void)hipHostFree(c->h_obj);
    if (c->h_bad) (void)hipHostFree(c->h_bad);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

extern "C" {

const char *lf_last_error(void) { return g_last_error.c_str(); }

lf_status lf_em_init(lf_ctx **out, const lf_params *p, const uint8_t *views, const float *S_P, const float *mu_T,
                     const float *q_warm, void *hip_stream) {
    g_last_error.clear();
    if (!out) return set_error(LF_EINVAL, "out is NULL");
    *out = nullptr;
    lf_status st = validate_params(p);
    if (st != LF_OK) return st;
    if (!views || !S_P || !mu_T) return set_error(LF_EINVAL, "views, S_P and mu_T are required");
    if (!(p->flags & LF_INPUTS_ON_DEVICE)) {
        st = validate_host_values(p, S_P, mu_T, q_warm);
        if (st != LF_OK) return st;
    }
    lf_ctx *c = new lf_ctx();
    c->p = *p;
    c->g = make_geometry(p);
    c->lambda = derived_lambda(p);
    if (hipGetDevice(&c->device) != hipSuccess) {
        ctx_free(c);
        return set_error(LF_EDEVICE, "no HIP device");
    }
    c->stream = (hipStream_t)hip_stream;   // NULL: the device's null stream
    c->own_stream = false;
    st = ctx_alloc(c);
    if (st == LF_OK && hipMemsetAsync(c->bad, 0, 4, c->stream) != hipSuccess)
        st = set_error(LF_EDEVICE, "clear counter");
    if (st == LF_OK) st = ctx_load(c, views, S_P, mu_T, q_warm);
    if (st != LF_OK) {
        std::string msg = g_last_error;
        ctx_free(c);
        g_last_error = msg;
        return st;
    }
    *out = c;
    return LF_OK;
}

lf_status lf_em_load(lf_ctx *c, const uint8_t *views, const float *S_P, const float *mu_T, const float *q_warm) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    return ctx_load(c, views, S_P, mu_T, q_warm);
}

// After the stream has been synchronised: report a pending deferred value
// check of device inputs (and clear the sticky counter).
static lf_status deferred_check(lf_ctx *c) {
    if (!c->check_pending) return LF_OK;
    c->check_pending = false;
    // the count of every frame loaded since the last report
    LF_HIP(hipMemcpyAsync(c->h_bad, c->bad, 4, hipMemcpyDeviceToHost, c->stream), "copy counter");
    LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
    const uint32_t bad = *c->h_bad;
    if (!bad) return LF_OK;
    *c->h_bad = 0;
    LF_HIP(hipMemsetAsync(c->bad, 0, 4, c->stream), "clear counter");
    LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
    c->loaded = false;
    return set_error(LF_EINVAL, "%u input values invalid in frames loaded since the last check (S_P outside [0,1], "
                                "mu_T not finite or q_warm outside [0,1])", bad);
}

static lf_status iterate(lf_ctx *c, int32_t n_iters, double *objective, unsigned long long *sweep) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    if (n_iters < 0) return set_error(LF_EINVAL, "n_iters=%d < 0", n_iters);
    if (!c->loaded) return set_error(LF_ESTATE, "no frame loaded");
    EmArgs a = make_em_args(&c->p, c->g, c->lambda);
    a.sweep_count = sweep;
    a.feat = c->feat;
    a.rho = c->rho;
    a.omr = c->omr;
    a.mu_T = c->mu_dev;
    a.q = c->q;
    a.d_idx = c->d_idx;
    a.lpix = c->lpix;
    a.obj = c->obj;
    if (c->dyn.span) {
        a.items = c->dyn_items;
        a.n_items = c->dyn_n;
    }
    int done = 0;
    while (done < n_iters) {
        const int n = std::min(kMaxItersPerLaunch, n_iters - done);
        a.n_iters = n;
        a.seed_from_d = (c->iters + done) > 0;   // start the sweep at the last level
        a.want_obj = objective != nullptr;      // else only the last iteration's (kept as L_pix)
        LF_HIP(launch_em(&c->p, c->g, a, c->tile, c->lds, c->stream, &c->dyn), "EM launch");
        if (objective) {
            LF_HIP(hipMemcpyAsync(c->h_obj, c->obj, (size_t)n * c->n_blocks * 8, hipMemcpyDeviceToHost, c->stream),
                   "copy objective");
            LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
            lf_status st = deferred_check(c);
            if (st != LF_OK) return st;
            for (int t = 0; t < n; ++t) {
                double s = 0.0;
                const double *row = c->h_obj + (size_t)t * c->n_blocks;
                for (int b = 0; b < c->n_blocks; ++b) s += row[b];
                objective[done + t] = s;
            }
        }
        done += n;
    }
    c->iters += n_iters;
    return LF_OK;
}

lf_status lf_em_iterate(lf_ctx *c, int32_t n_iters, double *objective) { return iterate(c, n_iters, objective, nullptr); }

lf_status lf_em_sweep_count(lf_ctx *c, int32_t n_iters, uint64_t *level_steps) {
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    if (!level_steps) return set_error(LF_EINVAL, "level_steps is NULL");
    LF_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(c->sweep), 2, 0u, c->stream), "clear counter");
    lf_status st = iterate(c, n_iters, nullptr, c->sweep);
    if (st != LF_OK) return st;
    unsigned long long v = 0;
    LF_HIP(hipMemcpyAsync(&v, c->sweep, sizeof v, hipMemcpyDeviceToHost, c->stream), "copy counter");
    LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
    *level_steps = v;
    return deferred_check(c);
}

lf_status lf_em_check(lf_ctx *c) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return deferred_check(c);
}

static lf_status copy_out(lf_ctx *c, void *dst, const void *src, size_t bytes) {
    const hipMemcpyKind kind = (c->p.flags & LF_OUTPUTS_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    LF_HIP(hipMemcpyAsync(dst, src, bytes, kind, c->stream), "copy output");
    return LF_OK;
}

lf_status lf_refocus(lf_ctx *c, float *rgb, int32_t *d_idx, float *q, uint8_t *hole, int32_t median) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    if (!rgb) return set_error(LF_EINVAL, "rgb is required");
    if (median != 0 && median != 3) return set_error(LF_EINVAL, "median=%d must be 0 or 3", median);
    if (!c->loaded || c->iters == 0) return set_error(LF_ESTATE, "refocus needs at least one EM iteration");
    const lf_params &p = c->p;
    const size_t HW = (size_t)p.H * p.W;
    const bool dev_out = p.flags & LF_OUTPUTS_ON_DEVICE;
    // device outputs: the refocus pass writes the level and weights too
    LF_HIP(launch_refocus_frame(&p, c->g, c->views, c->d_idx, c->q, c->rho, dev_out ? rgb : c->rgb,
                                dev_out ? hole : c->hole, c->rgb_med, median, dev_out ? d_idx : nullptr,
                                dev_out ? q : nullptr, c->stream),
           "refocus launch");
    lf_status st = LF_OK;
    if (!dev_out) {
        if (st == LF_OK) st = copy_out(c, rgb, c->rgb, HW * 12);
        if (st == LF_OK && hole) st = copy_out(c, hole, c->hole, HW);
    }
    if (!dev_out) {
        if (st == LF_OK && d_idx) st = copy_out(c, d_idx, c->d_idx, HW * 4);
        if (st == LF_OK && q) st = copy_out(c, q, c->q, HW * p.K * 4);
    }
    if (st != LF_OK) return st;
    if (!dev_out) {
        LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
        return deferred_check(c);
    }
    return LF_OK;
}

lf_status lf_segmentation_maps(lf_ctx *c, uint8_t *labels) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    if (!labels) return set_error(LF_EINVAL, "labels is required");
    if (!c->loaded || c->iters == 0) return set_error(LF_ESTATE, "segmentation maps need at least one EM iteration");
    const lf_params &p = c->p;
    if (p.W > 65535 || p.D > 32767) return set_error(LF_EINVAL, "segmentation maps need W <= 65535 and D <= 32767");
    const size_t KHW = (size_t)p.K * p.H * p.W;
    const bool dev_out = p.flags & LF_OUTPUTS_ON_DEVICE;
    SegArgs a{};
    a.d_idx = c->d_idx;
    a.q = c->q;
    a.keys = c->seg_keys;
    a.labels = dev_out ? labels : c->seg_labels;
    a.K = p.K;
    a.H = p.H;
    a.W = p.W;
    a.frac = c->g.frac;
    a.dmin_i = c->g.dmin_i;
    a.dstep_i = c->g.dstep_i;
    a.d_min = p.d_min;
    a.d_step = p.d_step;
    for (int k = 0; k < p.K; ++k) {
        a.bi[k] = c->g.bi[k];
        a.b[k] = p.baselines[k];
    }
    hipLaunchKernelGGL(lf_fill_i32_kernel, dim3((unsigned)((KHW + 255) / 256)), dim3(256), 0, c->stream, c->seg_keys,
                       KHW, -1);
    LF_HIP(hipGetLastError(), "segmentation fill launch");
    const dim3 grid((p.W + 255) / 256, p.H, p.K);
    hipLaunchKernelGGL(lf_seg_scatter_kernel, grid, dim3(256), 0, c->stream, a);
    LF_HIP(hipGetLastError(), "segmentation scatter launch");
    hipLaunchKernelGGL(lf_seg_resolve_kernel, grid, dim3(256), 0, c->stream, a);
    LF_HIP(hipGetLastError(), "segmentation resolve launch");
    if (!dev_out) {
        lf_status st = copy_out(c, labels, c->seg_labels, KHW);
        if (st != LF_OK) return st;
        LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
        return deferred_check(c);
    }
    return LF_OK;
}

lf_status lf_em_state(lf_ctx *c, float *q, int32_t *d_idx, float *L_pix) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    if (!c->loaded) return set_error(LF_ESTATE, "no frame loaded");
    if ((d_idx || L_pix) && c->iters == 0) return set_error(LF_ESTATE, "no EM iteration since the last load");
    const size_t HW = (size_t)c->p.H * c->p.W;
    lf_status st = LF_OK;
    if (q) st = copy_out(c, q, c->q, HW * c->p.K * 4);
    if (st == LF_OK && d_idx) st = copy_out(c, d_idx, c->d_idx, HW * 4);
    if (st == LF_OK && L_pix) st = copy_out(c, L_pix, c->lpix, HW * 4);
    if (st != LF_OK) return st;
    if (!(c->p.flags & LF_OUTPUTS_ON_DEVICE)) {
        LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
        return deferred_check(c);
    }
    return LF_OK;
}

lf_status lf_em_intermediates(lf_ctx *c, void *feat, float *rho) {
    g_last_error.clear();
    if (!c) return set_error(LF_EINVAL, "context is NULL");
    if (!c->loaded) return set_error(LF_ESTATE, "no frame loaded");
    const size_t KHW = (size_t)c->p.H * c->p.W * c->p.K;
    lf_status st = LF_OK;
    if (feat) st = copy_out(c, feat, c->feat, KHW * pair_bytes(c->p.storage));
    if (st == LF_OK && rho) st = copy_out(c, rho, c->rho, KHW * 4);
    if (st != LF_OK) return st;
    if (!(c->p.flags & LF_OUTPUTS_ON_DEVICE)) {
        LF_HIP(hipStreamSynchronize(c->stream), "synchronize");
        return deferred_check(c);
    }
    return LF_OK;
}

void lf_em_destroy(lf_ctx *c) { ctx_free(c); }

}  // extern "C"
