// Per-frame kernels around the EM iterations (gfx950):
//   lf_load_kernel         3x3 Sobel responses of R+G+B (Sec. III-C), and S_P
//                          of each view at the ray footprint of mu_T, its
//                          complement and the thresholded first weights
//                          (Sec. III-B, III-F), in one launch
//   lf_refocus_kernel      mean of the static rays (Eq. 2)
//   lf_median3_kernel      3x3 per-channel median of the refocused image (Sec. III-E)
//   lf_seg_*_kernel        per-view segmentation maps in each view's own grid (Sec. III-D)
// Included by one translation unit only.
#pragma once

#include "lf_em_kernels.h"

namespace lfem {

// ---------------------------------------------------------------------------
// Load pass: the descriptors and the ray prior of a frame in one launch.
// grid (ceil(W/256), ceil(H/kDescRows) + H, K), block 256: the blocks with
// blockIdx.y below ceil(H/kDescRows) compute descriptors, the others the
// ray prior of one row each (the two parts are independent).
// ---------------------------------------------------------------------------

// Descriptors of view k, rows y0 .. y0 + kDescRows - 1, columns x0 .. x0 +
// 255: the block stages the intensity sums L = R+G+B of its rows plus one
// row and one column of border on each side (replicated) in LDS, then every
// lane takes the 3x3 Sobel responses of its column down the rows.
constexpr int kDescRows = 8;

template <int ST>
__device__ __forceinline__ void descriptors_block(const uint8_t *__restrict__ views,
                                                  typename Pair<ST>::T *__restrict__ feat, int H, int W, int k,
                                                  int y0, int x0) {
    __shared__ int16_t L[kDescRows + 2][256 + 2];
    const int tid = threadIdx.x;
    const uint8_t *v = views + (size_t)k * H * W * 3;
    for (int i = tid; i < (kDescRows + 2) * 258; i += 256) {
        const int r = i / 258, c = i - r * 258;
        const int yy = clampi(y0 + r - 1, 0, H - 1), xx = clampi(x0 + c - 1, 0, W - 1);
        const uint8_t *px = v + ((size_t)yy * W + xx) * 3;
        L[r][c] = (int16_t)((int)px[0] + (int)px[1] + (int)px[2]);
    }
    __syncthreads();
    const int x = x0 + tid;
    if (x >= W) return;
    const float s = 1.0f / 4096.0f;  // exact: |G| <= 3060
    for (int r = 0; r < kDescRows && y0 + r < H; ++r) {
        const int16_t *a = L[r] + tid, *b = L[r + 1] + tid, *c = L[r + 2] + tid;
        const int gx = (a[2] - a[0]) + 2 * (b[2] - b[0]) + (c[2] - c[0]);
        const int gy = (c[0] - a[0]) + 2 * (c[1] - a[1]) + (c[2] - a[2]);
        feat[((size_t)k * H + y0 + r) * W + x] = make_pair<ST>((float)gx * s, (float)gy * s);
    }
}

// Ray prior and first weights of view k, row y, columns x0 .. x0 + 255.
struct PriorArgs {
    const float *S_P, *mu_T, *q_warm;
    float *rho, *omr, *q;   // static prior, dynamic prior 1 - rho, weights
    uint32_t *bad;  // count of invalid input values (device-resident inputs only)
    int K, H, W, storage, check;
    float tau;
    float b[kMaxViews];
};

__device__ __forceinline__ void ray_prior_row(const PriorArgs &a, int k, int y, int x0) {
    const int x = x0 + threadIdx.x;
    if (x >= a.W) return;
    const size_t pix = (size_t)y * a.W + x;
    const size_t i = (size_t)k * a.H * a.W + pix;
    const float mu = a.mu_T[pix];
    const float *row = a.S_P + ((size_t)k * a.H + y) * a.W;
    float r, om;
    ray_prior_value(row, a.W, x, a.b[k], mu, a.storage, r, om);
    a.rho[i] = r;
    a.omr[i] = om;
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

template <int ST>
__global__ __launch_bounds__(256) void lf_load_kernel(const uint8_t *__restrict__ views,
                                                      typename Pair<ST>::T *__restrict__ feat, PriorArgs a) {
    const int nd = (a.H + kDescRows - 1) / kDescRows;
    const int k = blockIdx.z, by = blockIdx.y, x0 = blockIdx.x * 256;
    if (by < nd) descriptors_block<ST>(views, feat, a.H, a.W, k, by * kDescRows, x0);
    else ray_prior_row(a, k, by - nd, x0);
}

// ---------------------------------------------------------------------------
// Dynamic-only work list (reconstruction of the dynamic reference pixels
// only, rho_ref < tau).  A work item is one wave: the next up to 64 dynamic
// pixels of a row that lie within `span` columns of the item's first one
// (span = a.seg_w, a multiple of 64, so that the item's view windows fit the
// LDS), cut greedily from left to right.  With the shared sweep (split) an
// item also holds at most kItemUnbounded pixels whose first sweep the prior
// bound is predicted to leave unbounded (seed_bounded): the wave shares an
// unbounded pixel's levels among lanes, cp = 64 / (their number) per pixel,
// so an item with many of them sweeps whole level ranges, and it sets the
// launch's time (the items all start at once).  A row of W columns then has
// at most floor(W/64) items of 64 pixels, floor((W-1)/span) closed by the
// span and one last item, plus, with split, at most W/64 closed by the
// unbounded limit (a budget: the limit is not applied beyond it), which
// per_row bounds.  grid H, one wave per row: the row's items (first column,
// number of pixels) and their number; the pixels not reconstructed take
// the level nearest mu_T and objective 0.
// ---------------------------------------------------------------------------
constexpr int kItemUnbounded = 16;

__device__ __forceinline__ float2 load_pair(const void *feat, int storage, size_t i) {
    if (storage == 0) return reinterpret_cast<const float2 *>(feat)[i];
    if (storage == 1) return widen(reinterpret_cast<const __half2 *>(feat)[i]);
    return widen(reinterpret_cast<const uint32_t *>(feat)[i]);
}

// Whether the prior bound leaves the first sweep of pixel (x, y) bounded:
// its energy at the first seed (the level nearest mu_T, the weights the
// frame was loaded with), in one-pass form from the descriptors in HBM,
// against prior_interval.  A prediction of the sweep's own test, which
// takes the exact energy from LDS; integer shifts.
__device__ __forceinline__ bool seed_bounded(const EmArgs &a, int K, int storage, int y, int x) {
    const size_t HW = (size_t)a.H * a.W, pix = (size_t)y * a.W + x;
    const float mu = a.mu_T[pix];
    const int j = nearest_level(a, mu);
    float Q = 0.0f;
    for (int k = 0; k < K; ++k) Q += a.q[(size_t)a.perm[k] * HW + pix];
    const bool empty = !(Q > 0.0f);
    float Wt = 0.0f, Ax = 0.0f, Ay = 0.0f, S = 0.0f;
    for (int k = 0; k < K; ++k) {
        const float w = empty ? 1.0f : a.q[(size_t)a.perm[k] * HW + pix];
        const int u = clampi(x - a.bi[k] * (a.dmin_i + j * a.dstep_i), 0, a.W - 1);
        const float2 f = load_pair(a.feat, storage, ((size_t)a.perm[k] * a.H + y) * a.W + u);
        Wt += w;
        Ax = fmaf(w, f.x, Ax);
        Ay = fmaf(w, f.y, Ay);
        S = fmaf(w, fmaf(f.x, f.x, f.y * f.y), S);
    }
    const float cw = empty ? 0.0f : a.beta_p;
    const float C = fmaxf(S - (Ax * Ax + Ay * Ay) / Wt, 0.0f);
    const float E = fmaf(cw, C, -log_prior(a, j, mu));
    int jl, jh;
    return prior_interval(a, E, mu, jl, jh);
}

// items of row y: items_row[2 i] = first column, items_row[2 i + 1] = pixels
__global__ __launch_bounds__(64) void lf_dyn_rows_kernel(EmArgs a, int per_row, int K, int storage, int split,
                                                         int *__restrict__ counts, int *__restrict__ rows) {
    const int y = blockIdx.x, lane = threadIdx.x;
    const float *rho_ref = a.rho + (size_t)a.perm[0] * a.H * a.W + (size_t)y * a.W;
    int *items_row = rows + (size_t)y * per_row * 2;
    const int budget = split ? a.W / 64 : 0;
    int n_items = 0, first = 0, n = 0, nu = 0, used = 0;   // wave-uniform
    auto close = [&]() {
        if (lane == 0 && n_items < per_row) {
            items_row[2 * n_items] = first;
            items_row[2 * n_items + 1] = n;
        }
        ++n_items;
    };
    for (int c0 = 0; c0 < a.W; c0 += 64) {
        const int col = c0 + lane;
        const bool in = col < a.W;
        const bool dyn = in && rho_ref[col] < a.tau;
        if (in && !dyn) {
            const size_t pix = (size_t)y * a.W + col;
            a.d_idx[pix] = nearest_level(a, a.mu_T[pix]);
            a.lpix[pix] = 0.0f;
        }
        const bool unb = split && dyn && !seed_bounded(a, K, storage, y, col);
        uint64_t m = __ballot(dyn);
        const uint64_t um = __ballot(unb);
        while (m) {
            const int b = __builtin_ctzll(m);
            const int cb = c0 + b;
            m &= m - 1;
            const bool u = (um >> b) & 1ull;
            if (n > 0) {
                const bool full = n == 64 || cb - first >= a.seg_w;
                const bool by_unb = !full && u && nu == kItemUnbounded && used < budget;
                if (full || by_unb) {
                    close();
                    used += by_unb ? 1 : 0;
                    n = 0;
                    nu = 0;
                }
            }
            if (n == 0) first = cb;
            ++n;
            nu += u ? 1 : 0;
        }
    }
    if (n > 0) close();
    if (lane == 0) counts[y] = min(n_items, per_row);
}

// One block: exclusive scan of the rows' item counts, then the list in row
// order as (row, first column, pixels).
__global__ __launch_bounds__(256) void lf_dyn_items_kernel(const int *__restrict__ counts,
                                                           const int *__restrict__ rows, int H, int per_row,
                                                           int4 *__restrict__ items, int *__restrict__ n_items) {
    __shared__ int part[256];
    const int t = threadIdx.x, per = (H + 255) / 256;
    const int beg = min(t * per, H), end = min(beg + per, H);
    int sum = 0;
    for (int y = beg; y < end; ++y) sum += counts[y];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int i = 0; i < 256; ++i) {
            const int v = part[i];
            part[i] = acc;
            acc += v;
        }
        *n_items = acc;
    }
    __syncthreads();
    int off = part[t];
    for (int y = beg; y < end; ++y) {
        const int c = counts[y];
        const int *r = rows + (size_t)y * per_row * 2;
        for (int i = 0; i < c; ++i) items[off++] = make_int4(y, r[2 * i], r[2 * i + 1], 0);
    }
}

// ---------------------------------------------------------------------------
// Refocus (Eq. 2).  grid (ceil(W/blockDim), H).
// ---------------------------------------------------------------------------
struct RefocusArgs {
    const uint8_t *views;
    const int32_t *d_idx;
    const float *q;
    const float *rho_ref;   // ray prior of the reference view (dynamic-only), else null
    float tau;
    float *rgb;
    uint8_t *hole;
    int32_t *d_out;         // device copies of the level and weights handed out, or null
    float *q_out;
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
    // the state handed out with the image, in the same pass
    if (a.d_out) a.d_out[pix] = a.d_idx[pix];
    if (a.q_out)
        for (int k = 0; k < a.K; ++k) a.q_out[k * HW + pix] = a.q[k * HW + pix];
    if (a.rho_ref && !(a.rho_ref[pix] < a.tau)) {
        // dynamic-only: a static reference ray shows the background itself
        const uint8_t *c_ref = a.views + (((size_t)a.ref * a.H + y) * a.W + x) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) a.rgb[pix * 3 + c] = (float)c_ref[c] / 255.0f;
        if (a.hole) a.hole[pix] = 0;
        return;
    }
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
            float t, omt;
            footprint_precise(x, a.b[k], d, i0, t, omt);
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


// ---------------------------------------------------------------------------
// Per-view segmentation maps (the updated segmentation of Sec. III-D, shown
// in each view's own pixel grid).  The ray of reference pixel (x, y) at its
// level lands in view k at u = x - b_k d, taken to the nearest pixel
// floor(u + 1/2); the ray with the largest level (the nearest surface) is
// the one seen.  keys [K][H][W] hold (level << 16 | x) of the ray seen, -1
// for none: an atomic max picks it independently of the order of arrival.
// Labels: 1 static (q >= 1/2), 0 dynamic, 2 no reference ray.
// ---------------------------------------------------------------------------
struct SegArgs {
    const int32_t *d_idx;
    const float *q;        // [K][H][W], array view order
    int32_t *keys;         // [K][H][W]
    uint8_t *labels;       // [K][H][W]
    int K, H, W, frac;
    int dmin_i, dstep_i;
    float d_min, d_step;
    int bi[kMaxViews];
    float b[kMaxViews];
};

__global__ __launch_bounds__(256) void lf_fill_i32_kernel(int32_t *p, size_t n, int32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Frame objective of each iteration from the EM kernel's FP64 block sums,
// summed in block order by one lane per iteration.
__global__ __launch_bounds__(64) void lf_objective_sum_kernel(const double *__restrict__ partials, int n_blocks,
                                                              int n, double *__restrict__ objective) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double *row = partials + (size_t)t * n_blocks;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += row[b];
    objective[t] = s;
}

// grid (ceil(W/256), H, K)
__global__ __launch_bounds__(256) void lf_seg_scatter_kernel(SegArgs a) {
    const int k = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.W) return;
    const int j = a.d_idx[(size_t)y * a.W + x];
    int u;
    if (!a.frac) {
        u = x - a.bi[k] * (a.dmin_i + j * a.dstep_i);
    } else {
        int i0;
        float t;
        footprint(x, a.b[k], fmaf((float)j, a.d_step, a.d_min), i0, t);
        u = i0 + (t >= 0.5f ? 1 : 0);
    }
    if (u < 0 || u >= a.W) return;
    atomicMax(&a.keys[((size_t)k * a.H + y) * a.W + u], (j << 16) | x);
}

// grid (ceil(W/256), H, K)
__global__ __launch_bounds__(256) void lf_seg_resolve_kernel(SegArgs a) {
    const int k = blockIdx.z, y = blockIdx.y;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= a.W) return;
    const size_t row = ((size_t)k * a.H + y) * a.W;
    const int32_t key = a.keys[row + u];
    uint8_t l = 2;
    if (key >= 0) l = a.q[row + (key & 0xffff)] >= 0.5f ? 1 : 0;
    a.labels[row + u] = l;
}

}  // namespace lfem
